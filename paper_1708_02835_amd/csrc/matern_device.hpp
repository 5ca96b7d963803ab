// Device evaluation of the Matérn covariance, Sec. 2.2 Eq. (2):
//   C(r; θ) = θ1 / (2^(θ3-1) Γ(θ3)) · (r/θ2)^θ3 · K_θ3(r/θ2),  C(0) = θ1.
//
// K_ν for arbitrary real ν > 0 follows Temme's method (N. M. Temme, J. Comput.
// Phys. 19 (1975) 324-337): write ν = μ + nl with |μ| <= 1/2, obtain K_μ and
// K_μ+1, then recur upward in order with K_a+1 = K_a-1 + (2a/x) K_a, which is
// stable for K.
//   * x <= 2: Temme's power series in (x/2)^2, whose leading coefficient uses
//     Γ1(μ) = (1/Γ(1-μ) - 1/Γ(1+μ)) / (2μ) and Γ2(μ) = (1/Γ(1-μ) + 1/Γ(1+μ)) / 2,
//     both taken from the Taylor series of 1/Γ(1+z) so that μ -> 0 has no
//     cancellation.
//   * x > 2: the representation K_μ(x) = sqrt(π) (2x)^μ e^-x U(μ+1/2, 2μ+1, 2x)
//     with the confluent hypergeometric function U.  The values z_k =
//     U(μ+1/2+k, 2μ+1, 2x) obey z_k-1 = 2(k+x) z_k - ((k+1/2)^2 - μ^2) z_k+1,
//     are the minimal solution of that recurrence (so Miller's backward
//     recurrence finds their ratios), and satisfy the normalisation
//     Σ_k [(μ+1/2)_k (1/2-μ)_k / k!] z_k = (2x)^-(μ+1/2), which follows from the
//     Laplace integral of U and the binomial series.  Hence
//     K_μ = sqrt(π/(2x)) e^-x / S with S = Σ_k c_k z_k / z_0, and
//     K_μ+1 = K_μ (μ + 1/2 + x - (1/4 - μ^2) z_1/z_0) / x.
//     The recurrence depth needed for binary64 accuracy falls like 1/x.
// Half-integer smoothness 1/2, 3/2, 5/2 uses the elementary closed forms
// (Sec. 2.2 names the exponential model for θ3 = 1/2).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "rgamma_table.hpp"

namespace gl {

struct MaternSetup {
    double theta1, theta2, nu;
    double mu;     // ν - nl, |μ| <= 1/2
    double pref;   // θ1 · 2^(1-ν) / Γ(ν)
    double g1, g2; // Temme Γ1(μ), Γ2(μ)
    double rgp;    // 1/Γ(1+μ)
    double rgm;    // 1/Γ(1-μ)
    double fact;   // μπ / sin(μπ)
    int nl;        // number of upward recurrence steps
    int kind;      // 0: general ν, 1: ν = 1/2, 2: ν = 3/2, 3: ν = 5/2
};

__host__ __device__ inline MaternSetup matern_setup(double t1, double t2, double t3)
{
    MaternSetup s;
    s.theta1 = t1;
    s.theta2 = t2;
    s.nu = t3;
    s.kind = (t3 == 0.5) ? 1 : (t3 == 1.5) ? 2 : (t3 == 2.5) ? 3 : 0;
    int nl = (int)floor(t3 + 0.5);
    double mu = t3 - nl;
    s.nl = nl;
    s.mu = mu;
    // even and odd parts of 1/Γ(1+z) at z = μ
    double m2 = mu * mu, ev = 0.0, od = 0.0;
    for (int k = GL_RGAMMA_TERMS - 2; k >= 0; k -= 2) ev = ev * m2 + gl_rgamma_coef[k];
    for (int k = GL_RGAMMA_TERMS - 1; k >= 1; k -= 2) od = od * m2 + gl_rgamma_coef[k];
    s.g2 = ev;
    s.g1 = -od;
    s.rgp = ev + mu * od;  // Σ c_k μ^k
    s.rgm = ev - mu * od;  // Σ c_k (-μ)^k
    double pm = M_PI * mu;
    if (fabs(pm) < 1e-4) {
        double p2 = pm * pm;
        s.fact = 1.0 + p2 / 6.0 + 7.0 * p2 * p2 / 360.0;
    } else {
        s.fact = pm / sin(pm);
    }
    // Γ(ν) from Γ(1+μ) = 1/rgp: Γ(μ+nl) = Γ(1+μ) Π_{j=1}^{nl-1} (μ+j); nl = 0 → Γ(μ) = Γ(1+μ)/μ
    double gnu;
    if (nl == 0) {
        gnu = 1.0 / (s.rgp * mu);
    } else {
        gnu = 1.0 / s.rgp;
        for (int j = 1; j < nl; ++j) gnu *= (mu + j);
    }
    s.pref = t1 * exp2(1.0 - t3) / gnu;
    return s;
}

// Per-k constants of the series and the recurrence below, for one μ: filled
// once per workgroup in LDS so the per-element loops only multiply and add
// (1/(k-μ), 1/(k+μ) for the series, 1/k for both, and the recurrence
// coefficients (k+1/2)² - μ² and ((k-1/2)² - μ²)/k).
constexpr int GL_TEMME_TERMS = 40;
constexpr int GL_MILLER_MAX = 80;
struct BesselTab {
    double rm[GL_TEMME_TERMS];     // 1/(k - μ)
    double rp[GL_TEMME_TERMS];     // 1/(k + μ)
    double rk[GL_MILLER_MAX + 1];  // 1/k
    double ma[GL_MILLER_MAX + 1];  // (k + 1/2)² - μ²
    double mb[GL_MILLER_MAX + 1];  // ((k - 1/2)² - μ²) / k
};

// Every thread of the workgroup calls this before the first matern_eval with
// the table; it ends with a barrier.
__device__ inline void bessel_tab_init(const MaternSetup &s, BesselTab &t)
{
    for (int k = threadIdx.x; k <= GL_MILLER_MAX; k += blockDim.x) {
        const double dk = (double)k;
        if (k >= 1 && k < GL_TEMME_TERMS) {
            t.rm[k] = 1.0 / (dk - s.mu);
            t.rp[k] = 1.0 / (dk + s.mu);
        }
        t.rk[k] = k ? 1.0 / dk : 0.0;
        t.ma[k] = (dk + 0.5) * (dk + 0.5) - s.mu * s.mu;
        t.mb[k] = k ? ((dk - 0.5) * (dk - 0.5) - s.mu * s.mu) / dk : 0.0;
    }
    __syncthreads();
}

// K_μ(x) and K_μ+1(x) for x <= 2 (Temme's series), unscaled; lx = log(2/x).
// One exponential e^σ, σ = μ lx, gives sinh σ, cosh σ and (x/2)^∓μ.
__host__ __device__ inline void bessel_k_temme(const MaternSetup &s, double x, double lx, double &k0, double &k1,
                                               const BesselTab *tab = nullptr)
{
    const double mu = s.mu;
    const double sig = mu * lx;
    const double e = exp(sig), ei = 1.0 / e;
    double shs;  // sinh(σ)/σ
    if (fabs(sig) < 0.1) {
        const double q = sig * sig;  // Taylor series to σ⁸, remainder below 3e-18
        shs = 1.0 + q / 6.0 * (1.0 + q / 20.0 * (1.0 + q / 42.0 * (1.0 + q / 72.0)));
    } else {
        shs = 0.5 * (e - ei) / sig;
    }
    double f = s.fact * (0.5 * (e + ei) * s.g1 + shs * lx * s.g2);
    double p = 0.5 * e / s.rgp;   // ½ (x/2)^-μ Γ(1+μ)
    double q = 0.5 * ei / s.rgm;  // ½ (x/2)^μ Γ(1-μ)
    double c = 1.0;
    const double d = 0.25 * x * x;
    double sum0 = f, sum1 = p;
    const double mu2 = mu * mu;
    for (int k = 1; k < GL_TEMME_TERMS; ++k) {
        double dk = (double)k;
        if (tab) {
            const double rm = tab->rm[k], rp = tab->rp[k];
            f = (dk * f + p + q) * (rm * rp);
            c *= d * tab->rk[k];
            p *= rm;
            q *= rp;
        } else {
            f = (dk * f + p + q) / (dk * dk - mu2);
            c *= d / dk;
            p /= (dk - mu);
            q /= (dk + mu);
        }
        double t0 = c * f;
        double t1 = c * (p - dk * f);
        sum0 += t0;
        sum1 += t1;
        if (fabs(t0) < 1e-17 * fabs(sum0) && fabs(t1) < 1e-17 * fabs(sum1)) break;
    }
    k0 = sum0;
    k1 = sum1 * 2.0 / x;
}

// e^x K_μ(x) and e^x K_μ+1(x) for x > 2 (backward recurrence for U ratios).
__host__ __device__ inline void bessel_k_miller_scaled(const MaternSetup &s, double x, double &k0, double &k1,
                                                       const BesselTab *tab = nullptr)
{
    const double mu2 = s.mu * s.mu;
    int kmax = (int)(8.0 + 140.0 / x);
    if (kmax > GL_MILLER_MAX) kmax = GL_MILLER_MAX;
    double z1 = 0.0, z0 = 1.0;  // z_{K+1}, z_K
    double t = 1.0;             // Horner accumulation of Σ c_k z_k from the top
    for (int k = kmax; k >= 1; --k) {
        double dk = (double)k;
        double zm, ck;
        if (tab) {
            zm = 2.0 * (dk + x) * z0 - tab->ma[k] * z1;
            ck = tab->mb[k];
        } else {
            zm = 2.0 * (dk + x) * z0 - ((dk + 0.5) * (dk + 0.5) - mu2) * z1;
            ck = ((dk - 0.5) * (dk - 0.5) - mu2) / dk;
        }
        z1 = z0;
        z0 = zm;
        t = zm + ck * t;
    }
    double ssum = t / z0;
    double r0 = z1 / z0;
    k0 = sqrt(M_PI / (2.0 * x)) / ssum;
    k1 = k0 * (s.mu + 0.5 + x - (0.25 - mu2) * r0) / x;
}

// The half-integer closed forms at x = r/θ2 (s.kind 1, 2, 3).
__host__ __device__ inline double matern_closed(const MaternSetup &s, double x)
{
    switch (s.kind) {
    case 1: return s.theta1 * exp(-x);
    case 2: return s.theta1 * (1.0 + x) * exp(-x);
    default: return s.theta1 * (1.0 + x + x * x / 3.0) * exp(-x);
    }
}

// Matérn covariance at distance r for a half-integer setup (s.kind != 0):
// the same values as matern_eval, without the Bessel evaluator (so kernels
// that only take this path keep few registers).
__host__ __device__ inline double matern_eval_closed(const MaternSetup &s, double r)
{
    if (r == 0.0) return s.theta1;
    const double x = r / s.theta2;
    if (x > 2000.0) return 0.0;
    return matern_closed(s, x);
}

// Matérn covariance at distance r (r >= 0); tab (may be NULL) from
// bessel_tab_init for the same setup.
__host__ __device__ inline double matern_eval(const MaternSetup &s, double r, const BesselTab *tab = nullptr)
{
    if (r == 0.0) return s.theta1;
    const double x = r / s.theta2;
    // Past x = 2000 the correlation C/θ1 is below e^-1600 for every ν <= 50,
    // so C underflows to 0 for any finite θ1; returning early also keeps
    // the closed forms' polynomials and the recurrences below finite.
    if (x > 2000.0) return 0.0;
    if (s.kind != 0) return matern_closed(s, x);
    // Below 1e-150 the distance is far inside rounding of a repeated location;
    // the clamp keeps K_μ+1 (about x^-3/2 at most) and the scaled recurrence
    // below finite.
    const double xc = fmax(x, 1e-150);
    double ka, kb;
    const bool small = (xc <= 2.0);
    const double lgx = log(xc);  // serves the series' log(2/x) and x^ν or x^ν e^-x
    if (small) bessel_k_temme(s, xc, M_LN2 - lgx, ka, kb, tab);
    else bessel_k_miller_scaled(s, xc, ka, kb, tab);
    double knu;
    double lsc = 0.0;  // natural log of the power of two divided out of (ka, kb)
    if (s.nl == 0) {
        knu = ka;
    } else {
        // (ka, kb) = (K_μ+i-1, K_μ+i) → K_μ+nl.  K grows with the order, like
        // (2/x)^ν Γ(ν)/2 for small x, and overflows binary64 at large ν while
        // x^ν underflows; the pair is rescaled by 2^-900 whenever it passes
        // 2^500, so it stays below 2^124 after a rescale, one step multiplies
        // it by at most 1 + 2ν/x < 2^505 (ν <= 50, x >= 1e-150), and the
        // scale joins the exponent of x^ν at the end.
        const double xi = 1.0 / xc;
        if (kb > 0x1p500) {
            ka *= 0x1p-900;
            kb *= 0x1p-900;
            lsc += 900.0 * M_LN2;
        }
        for (int i = 1; i < s.nl; ++i) {
            double kc = ka + (2.0 * (s.mu + i) * xi) * kb;
            ka = kb;
            kb = kc;
            if (kb > 0x1p500) {
                ka *= 0x1p-900;
                kb *= 0x1p-900;
                lsc += 900.0 * M_LN2;
            }
        }
        knu = kb;
    }
    if (small) return s.pref * exp(s.nu * lgx + lsc) * knu;
    return s.pref * exp(s.nu * lgx - xc + lsc) * knu;
}

__host__ __device__ inline double dist2d(double x1, double y1, double x2, double y2)
{
    double dx = x1 - x2, dy = y1 - y2;
    return sqrt(dx * dx + dy * dy);
}

// Great-circle distance on a sphere of radius rho (Sec. 7.4): x = longitude,
// y = latitude in degrees; the haversine h = sin²(Δφ/2) + cos φ1 cos φ2
// sin²(Δλ/2) gives d = 2 rho asin(√h), h clamped to [0, 1].
__host__ __device__ inline double gcd_dist(double x1, double y1, double x2, double y2, double rho)
{
    const double deg = M_PI / 180.0;
    const double p1 = y1 * deg, p2 = y2 * deg;
    const double sp = sin(0.5 * (p2 - p1));
    const double sl = sin(0.5 * ((x2 - x1) * deg));
    double h = sp * sp + cos(p1) * cos(p2) * sl * sl;
    h = fmin(fmax(h, 0.0), 1.0);
    return 2.0 * rho * asin(sqrt(h));
}

__host__ __device__ inline double geo_dist(const Geom &g, double x1, double y1, double x2, double y2)
{
    return g.metric ? gcd_dist(x1, y1, x2, y2, g.radius) : dist2d(x1, y1, x2, y2);
}

}  // namespace gl
