/*
 * Reference oracle for the exact Gaussian log-likelihood with a Matérn
 * covariance (ExaGeoStat, arXiv 1708.02835).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the HIP implementation.
 *
 * Everything is plain, single-threaded IEEE binary64 C, compiled without
 * fused multiply-add contraction and without fast-math, written to be checked
 * against the paper by eye:
 *
 *   - Matérn covariance, Sec. 2.2 Eq. (2):
 *       C(r; θ) = θ1 / (2^(θ3-1) Γ(θ3)) · (r/θ2)^θ3 · K_θ3(r/θ2),  C(0) = θ1.
 *     The modified Bessel function of the second kind is taken from its
 *     integral representation K_ν(x) = ∫_0^∞ exp(-x cosh t) cosh(ν t) dt
 *     (DLMF 10.32.9), evaluated with the trapezoidal rule.  The paper names
 *     K_ν but gives no algorithm for it.
 *   - Cholesky factorisation Σ = L Lᵀ (Sec. 6.5, Alg. 2 step "dpotrf"),
 *     unblocked, row by row (Cholesky–Banachiewicz).
 *   - Forward substitution L w = Z (Alg. 2, "dtrsm").
 *   - log|Σ| = 2 Σ_i log L_ii (Sec. 6.1) and the dot product wᵀw (Alg. 2),
 *     both with Neumaier-compensated summation.
 *   - l(θ) = -n/2 log(2π) - ½ log|Σ| - ½ wᵀw (Sec. 2 Eq. (1), Alg. 2 last step).
 *   - Kriging Z1 = Σ12 Σ22⁻¹ Z2 (Sec. 2.3 Eq. (5), Alg. 3), and the
 *     prediction variance, the diagonal of Σ11 - Σ12 Σ22⁻¹ Σ21 (Eq. (4)),
 *     as θ1 - ‖L⁻¹ σ_k‖² with σ_k the k-th column of Σ21.
 *   - Synthetic field Z = L e (Sec. 6.4, Alg. 1).
 *   - Independent-blocks (IND) approximation (Sec. 6.8): every covariance
 *     between locations of different diagonal blocks is set to zero, so the
 *     log-likelihood is the sum of the exact log-likelihoods of the blocks of
 *     consecutive locations.
 *   - Distances: Euclidean in the plane (Sec. 2), or great-circle distance on
 *     a sphere of radius ρ by the haversine formula (Sec. 7.4, used for the
 *     longitude/latitude data): hav(d/ρ) = hav(Δφ) + cos φ1 cos φ2 hav(Δλ),
 *     hav(a) = sin²(a/2), with x = longitude and y = latitude in degrees.
 *
 * Matrices are dense row-major n×n arrays owned by the caller.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- K_ν ---- */

/*
 * e^x K_ν(x) = ∫_0^∞ exp(-x (cosh t - 1)) cosh(ν t) dt.
 *
 * The integrand is analytic and decays double-exponentially, so the
 * trapezoidal rule converges geometrically in 1/h (Trefethen & Weideman,
 * SIAM Review 56 (2014)).  For large x the integrand is a narrow bump of width
 * about 1/sqrt(x) around t = 0, so the step shrinks like 1/sqrt(x).  All terms
 * are positive: no cancellation.  The sum stops once a term is below e^-745
 * relative to the first one and t is past the bump.
 */
double oracle_bessel_k_scaled(double nu, double x)
{
    double h = 0.08;
    if (x > 0.0 && 0.4 / sqrt(x) < h) h = 0.4 / sqrt(x);
    double sum = 0.5; /* t = 0: exp(0) * cosh(0), trapezoid half weight */
    for (long k = 1;; ++k) {
        double t = (double)k * h;
        double e = -x * (cosh(t) - 1.0);
        if (e + nu * t < -745.0 && t > 1.0) break;
        sum += exp(e) * cosh(nu * t);
    }
    return h * sum;
}

double oracle_bessel_k(double nu, double x)
{
    return exp(-x) * oracle_bessel_k_scaled(nu, x);
}

/*
 * x^ν K_ν(x) = ∫_0^∞ exp(ν log x - x cosh t) cosh(ν t) dt, the same integral
 * with the power of x taken inside, by the same trapezoidal rule.  Each term
 * is formed as ½ (exp(a + ν t) + exp(a - ν t)), a = ν log x - x cosh t, so
 * neither x^ν (which underflows for large ν and small x) nor K_ν (which then
 * overflows) is formed on its own; the product stays near 2^(ν-1) Γ(ν).  The
 * log of the larger half, ν log x - x cosh t + ν t, is concave in t with its
 * peak where x sinh t = ν, so a term below e^-745 relative to the largest one
 * so far lies past the peak, and the sum stops there.
 */
double oracle_xnu_bessel_k(double nu, double x)
{
    double h = 0.08;
    if (x > 0.0 && 0.4 / sqrt(x) < h) h = 0.4 / sqrt(x);
    const double lx = log(x);
    double peak = nu * lx - x;
    double sum = 0.5 * exp(peak); /* t = 0, trapezoid half weight */
    for (long k = 1;; ++k) {
        double t = (double)k * h;
        double a = nu * lx - x * cosh(t);
        double top = a + nu * t;
        if (top > peak) peak = top;
        if (top < peak - 745.0 && t > 1.0) break;
        sum += 0.5 * (exp(a + nu * t) + exp(a - nu * t));
    }
    return h * sum;
}

/* Matérn covariance at distance r, Sec. 2.2 Eq. (2). */
double oracle_matern(double r, double theta1, double theta2, double theta3)
{
    if (r == 0.0) return theta1; /* limit of x^ν K_ν(x) as x → 0 is 2^(ν-1) Γ(ν) */
    double x = r / theta2;
    double pref = theta1 / (pow(2.0, theta3 - 1.0) * tgamma(theta3));
    return pref * oracle_xnu_bessel_k(theta3, x);
}

/* ---------------------------------------------------------- distances ---- */

/* metric 0: Euclidean distance in the plane (Sec. 2, d = 2).
 * metric 1: great-circle distance on a sphere of radius `radius` (Sec. 7.4),
 *           x = longitude, y = latitude, both in degrees; the haversine
 *           relation is solved for d as d = 2 ρ asin(√h), with h clamped to
 *           [0, 1] against rounding. */
double oracle_distance(int metric, double radius, double x1, double y1, double x2, double y2)
{
    if (metric == 0) {
        double dx = x1 - x2, dy = y1 - y2;
        return sqrt(dx * dx + dy * dy);
    }
    const double deg = M_PI / 180.0;
    double phi1 = y1 * deg, phi2 = y2 * deg;
    double dphi = phi2 - phi1, dlam = (x2 - x1) * deg;
    double s1 = sin(0.5 * dphi), s2 = sin(0.5 * dlam);
    double h = s1 * s1 + cos(phi1) * cos(phi2) * s2 * s2;
    if (h < 0.0) h = 0.0;
    if (h > 1.0) h = 1.0;
    return 2.0 * radius * asin(sqrt(h));
}

/* Dense n1×n2 row-major covariance between point sets 1 and 2
 * (genDistanceMatrix followed by genCovMatrix in Alg. 1-3). */
void oracle_cov_matrix(const double *x1, const double *y1, int64_t n1,
                       const double *x2, const double *y2, int64_t n2,
                       double theta1, double theta2, double theta3,
                       int metric, double radius, double *out)
{
    for (int64_t i = 0; i < n1; ++i)
        for (int64_t j = 0; j < n2; ++j)
            out[i * n2 + j] = oracle_matern(oracle_distance(metric, radius, x1[i], y1[i], x2[j], y2[j]),
                                            theta1, theta2, theta3);
}

/* Symmetric n×n covariance: lower triangle evaluated, mirrored above. */
void oracle_cov_symmetric(const double *x, const double *y, int64_t n,
                          double theta1, double theta2, double theta3,
                          int metric, double radius, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            double v = oracle_matern(oracle_distance(metric, radius, x[i], y[i], x[j], y[j]),
                                     theta1, theta2, theta3);
            out[i * n + j] = v;
            out[j * n + i] = v;
        }
}

/* ------------------------------------------------------------ Cholesky ---- */

/*
 * In-place Cholesky–Banachiewicz on a row-major n×n array: on return the lower
 * triangle holds L with Σ = L Lᵀ; the strict upper triangle is set to zero.
 * Returns 0, or j+1 when the j-th pivot (0-based) is not positive — the
 * LAPACK dpotrf "info" convention.
 */
int64_t oracle_cholesky(double *a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        double *li = a + i * n;
        for (int64_t j = 0; j <= i; ++j) {
            const double *lj = a + j * n;
            double s = li[j];
            for (int64_t k = 0; k < j; ++k) s -= li[k] * lj[k];
            if (i == j) {
                if (!(s > 0.0)) return j + 1;
                li[j] = sqrt(s);
            } else {
                li[j] = s / lj[j];
            }
        }
        for (int64_t j = i + 1; j < n; ++j) li[j] = 0.0;
    }
    return 0;
}

/* L w = z, L lower triangular row-major. */
void oracle_forward(const double *l, int64_t n, const double *z, double *w)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = z[i];
        for (int64_t k = 0; k < i; ++k) s -= l[i * n + k] * w[k];
        w[i] = s / l[i * n + i];
    }
}

/* Lᵀ v = w, L lower triangular row-major. */
void oracle_backward(const double *l, int64_t n, const double *w, double *v)
{
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = w[i];
        for (int64_t k = i + 1; k < n; ++k) s -= l[k * n + i] * v[k];
        v[i] = s / l[i * n + i];
    }
}

/* z = L e, L lower triangular row-major (Alg. 1, "dtrmm"). */
void oracle_trmv(const double *l, int64_t n, const double *e, double *z)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = 0; k <= i; ++k) s += l[i * n + k] * e[k];
        z[i] = s;
    }
}

/* Neumaier's compensated sum. */
static double neumaier_sum(const double *v, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + v[i];
        if (fabs(s) >= fabs(v[i])) c += (s - t) + v[i];
        else c += (v[i] - t) + s;
        s = t;
    }
    return s + c;
}

/* log|Σ| = 2 Σ log L_ii, summed as logs (Sec. 6.1 reads "product of the
 * diagonal"; the product itself under/overflows at realistic n). */
double oracle_logdet(const double *l, int64_t n)
{
    double *t = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) t[i] = 2.0 * log(l[i * n + i]);
    double r = neumaier_sum(t, n);
    free(t);
    return r;
}

double oracle_dot(const double *w, int64_t n)
{
    double *t = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) t[i] = w[i] * w[i];
    double r = neumaier_sum(t, n);
    free(t);
    return r;
}

/*
 * l(θ) by Alg. 2: Σ(θ) → L → w = L⁻¹ Z → logdet, wᵀw → l.
 * out[0] = l, out[1] = log|Σ|, out[2] = Zᵀ Σ⁻¹ Z.  Returns the Cholesky info
 * (0 on success); on failure out[0] = -inf and out[1], out[2] are NaN.
 * When l_out is not NULL the factor (row-major n×n) is copied there.
 */
int64_t oracle_loglik(const double *x, const double *y, const double *z, int64_t n,
                      double theta1, double theta2, double theta3, int metric, double radius,
                      double *out, double *l_out)
{
    double *a = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    oracle_cov_symmetric(x, y, n, theta1, theta2, theta3, metric, radius, a);
    int64_t info = oracle_cholesky(a, n);
    if (info != 0) {
        out[0] = -INFINITY;
        out[1] = NAN;
        out[2] = NAN;
    } else {
        oracle_forward(a, n, z, w);
        double logdet = oracle_logdet(a, n);
        double quad = oracle_dot(w, n);
        out[0] = -0.5 * quad - 0.5 * logdet - 0.5 * (double)n * log(2.0 * M_PI);
        out[1] = logdet;
        out[2] = quad;
    }
    if (l_out) memcpy(l_out, a, (size_t)n * (size_t)n * sizeof(double));
    free(a);
    free(w);
    return info;
}

/*
 * Kriging, Sec. 2.3 Eq. (5) with Alg. 3: X = Σ22⁻¹ Z2 through the Cholesky
 * factor (forward then backward substitution), then Z1 = Σ12 X.  When var is
 * not NULL, the prediction variances of Eq. (4): var_k = θ1 - uᵀu with
 * L u = σ_k, σ_k the covariances between new point k and the n observed
 * points (Σ11 has θ1 on its diagonal).  Returns the Cholesky info.
 */
int64_t oracle_krige(const double *x, const double *y, const double *z, int64_t n,
                     const double *xn, const double *yn, int64_t m,
                     double theta1, double theta2, double theta3, int metric, double radius,
                     double *znew, double *var)
{
    double *a = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    double *v = (double *)malloc((size_t)n * sizeof(double));
    double *sk = (double *)malloc((size_t)n * sizeof(double));
    oracle_cov_symmetric(x, y, n, theta1, theta2, theta3, metric, radius, a);
    int64_t info = oracle_cholesky(a, n);
    if (info == 0) {
        oracle_forward(a, n, z, w);
        oracle_backward(a, n, w, v);
        for (int64_t k = 0; k < m; ++k) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                sk[j] = oracle_matern(oracle_distance(metric, radius, xn[k], yn[k], x[j], y[j]),
                                      theta1, theta2, theta3);
                s += sk[j] * v[j];
            }
            znew[k] = s;
            if (var) {
                oracle_forward(a, n, sk, w);
                var[k] = theta1 - oracle_dot(w, n);
            }
        }
    }
    free(a);
    free(w);
    free(v);
    free(sk);
    return info;
}

/* Synthetic measurements, Sec. 6.4 Alg. 1: Σ(θ) = L Lᵀ, Z = L e.
 * Returns the Cholesky info. */
int64_t oracle_synth(const double *x, const double *y, const double *e, int64_t n,
                     double theta1, double theta2, double theta3, int metric, double radius,
                     double *z)
{
    double *a = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    oracle_cov_symmetric(x, y, n, theta1, theta2, theta3, metric, radius, a);
    int64_t info = oracle_cholesky(a, n);
    if (info == 0) oracle_trmv(a, n, e, z);
    free(a);
    return info;
}

/*
 * IND approximation, Sec. 6.8: Σ with every off-diagonal block annihilated is
 * block diagonal, with diagonal blocks of `block` consecutive locations (the
 * last one shorter when block does not divide n); its log-likelihood is the
 * sum over the blocks of Eq. (1) for the block alone.  out[0..2] as for
 * oracle_loglik (sums over blocks).  Returns 0, or the 1-based global column
 * of the first non-positive pivot.
 */
int64_t oracle_loglik_ind(const double *x, const double *y, const double *z, int64_t n,
                          double theta1, double theta2, double theta3, int metric, double radius,
                          int64_t block, double *out)
{
    double l = 0.0, ld = 0.0, q = 0.0;
    for (int64_t s = 0; s < n; s += block) {
        const int64_t m = (n - s < block) ? n - s : block;
        double part[3];
        int64_t info = oracle_loglik(x + s, y + s, z + s, m, theta1, theta2, theta3, metric, radius, part, NULL);
        if (info != 0) {
            out[0] = -INFINITY;
            out[1] = NAN;
            out[2] = NAN;
            return s + info;
        }
        l += part[0];
        ld += part[1];
        q += part[2];
    }
    out[0] = l;
    out[1] = ld;
    out[2] = q;
    return 0;
}

/*
 * Kriging under the IND approximation (Sec. 6.8 applied to the prediction of
 * Sec. 2.3 Eq. (5)): the covariance of all n locations, observed and
 * held-out alike, keeps only its diagonal blocks of `block` consecutive
 * locations (the last one shorter), so the blocks are independent fields and
 * each held-out value is predicted from the observed values of its own block:
 * Z_M = Σ_MO Σ_OO⁻¹ Z_O within the block (zero when the block observes
 * nothing).  miss[i] != 0 marks location i as held out; znew receives the
 * predictions in location order (one per held-out location).  Returns 0, or
 * the 1-based index, among all n locations, of the observed location whose
 * pivot is not positive.
 */
int64_t oracle_krige_ind(const double *x, const double *y, const double *z, const int32_t *miss, int64_t n,
                         double theta1, double theta2, double theta3, int metric, double radius,
                         int64_t block, double *znew)
{
    double *a = (double *)malloc((size_t)block * (size_t)block * sizeof(double));
    double *bx = (double *)malloc((size_t)block * sizeof(double));
    double *by = (double *)malloc((size_t)block * sizeof(double));
    double *bz = (double *)malloc((size_t)block * sizeof(double));
    double *w = (double *)malloc((size_t)block * sizeof(double));
    double *v = (double *)malloc((size_t)block * sizeof(double));
    int64_t *gi = (int64_t *)malloc((size_t)block * sizeof(int64_t));
    int64_t info = 0, out = 0;
    for (int64_t s = 0; s < n && info == 0; s += block) {
        const int64_t e = (n - s < block) ? n : s + block;
        int64_t no = 0;
        for (int64_t i = s; i < e; ++i)
            if (!miss[i]) {
                bx[no] = x[i];
                by[no] = y[i];
                bz[no] = z[i];
                gi[no] = i;
                ++no;
            }
        if (no > 0) {
            oracle_cov_symmetric(bx, by, no, theta1, theta2, theta3, metric, radius, a);
            const int64_t bi = oracle_cholesky(a, no);
            if (bi != 0) {
                info = gi[bi - 1] + 1;
                break;
            }
            oracle_forward(a, no, bz, w);
            oracle_backward(a, no, w, v);
        }
        for (int64_t i = s; i < e; ++i) {
            if (!miss[i]) continue;
            double acc = 0.0;
            for (int64_t j = 0; j < no; ++j)
                acc += oracle_matern(oracle_distance(metric, radius, x[i], y[i], bx[j], by[j]), theta1, theta2,
                                     theta3) * v[j];
            znew[out++] = acc;
        }
    }
    free(a);
    free(bx);
    free(by);
    free(bz);
    free(w);
    free(v);
    free(gi);
    return info;
}
