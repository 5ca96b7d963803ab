// Σ(θ) generation kernels (Alg. 1 steps 3-4, Alg. 2 step 2, Alg. 3 steps 3-6):
// the distance matrix is never stored; each element is evaluated from the two
// locations and written once.
#include "batch.hpp"
#include "common.hpp"
#include "matern_device.hpp"
#include "mfma.hpp"

namespace gl {

// Decode a packed lower-triangle tile index t into (i, j), i >= j.
__device__ inline void tile_from_index(int64_t t, int64_t &i, int64_t &j)
{
    int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    i = r;
    j = t - r * (r + 1) / 2;
}

// One workgroup per tile: all b×b entries of tile (i, j) of the packed lower
// storage.  Rows and columns at or beyond n are padding: 1 on the global
// diagonal, 0 elsewhere, so the padded matrix is block-diagonal with an
// identity tail and the likelihood terms of the first n rows are unchanged.
// Diagonal tiles are written in full (both triangles).  Stores are coalesced:
// consecutive threads write consecutive rows of one column.  When norm2 is not
// NULL, the tile's squared Frobenius norm is written to norm2[t] by a
// fixed-order block reduction.
// MODE (checked by the launchers): GEN_ANY any distance and smoothness;
// GEN_EUCLID Euclidean distance, so the kernel carries no great-circle
// trigonometry; GEN_CLOSED Euclidean distance and smoothness 1/2, 3/2 or
// 5/2, so it carries no Bessel evaluator either.  Fewer registers let more
// waves share a CU; the values are the same, bit for bit, in every mode.
enum { GEN_ANY = 0, GEN_EUCLID = 1, GEN_CLOSED = 2 };

template <int B, int MODE>
__device__ __forceinline__ void gen_tiles_body(double *__restrict__ tiles, const double *__restrict__ x,
                                               const double *__restrict__ y, int64_t n, gl_theta th, Geom geo,
                                               double *__restrict__ norm2, int64_t t)
{
    int64_t ti, tj;
    tile_from_index(t, ti, tj);
    const MaternSetup ms = matern_setup(th.theta1, th.theta2, th.theta3);
    __shared__ double xcs[B], ycs[B];  // the tile's column locations
    for (int c = threadIdx.x; c < B; c += 256) {
        const int64_t gc = tj * B + c;
        xcs[c] = gc < n ? x[gc] : 0.0;
        ycs[c] = gc < n ? y[gc] : 0.0;
    }
    const BesselTab *tabp = nullptr;
    if constexpr (MODE == GEN_CLOSED) {
        __syncthreads();
    } else {
        __shared__ BesselTab tab;
        bessel_tab_init(ms, tab);  // ends with the barrier the staging needs too
        tabp = &tab;
    }
    double *T = tiles + t * (int64_t)B * B;
    constexpr int RPT = (B + 255) / 256;
    double xr[RPT], yr[RPT];
    int64_t gr[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        int r = threadIdx.x + 256 * q;
        gr[q] = ti * B + r;
        bool ok = (r < B) && gr[q] < n;
        xr[q] = ok ? x[gr[q]] : 0.0;
        yr[q] = ok ? y[gr[q]] : 0.0;
    }
    double ss = 0.0;
    for (int c = 0; c < B; ++c) {
        const int64_t gc = tj * B + c;
        const bool colok = gc < n;
        const double xc = xcs[c];
        const double yc = ycs[c];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int r = threadIdx.x + 256 * q;
            if (r >= B) continue;
            double v;
            if (colok && gr[q] < n) {
                if constexpr (MODE == GEN_CLOSED) v = matern_eval_closed(ms, dist2d(xr[q], yr[q], xc, yc));
                else if constexpr (MODE == GEN_EUCLID) v = matern_eval(ms, dist2d(xr[q], yr[q], xc, yc), tabp);
                else v = matern_eval(ms, geo_dist(geo, xr[q], yr[q], xc, yc), tabp);
            } else {
                v = (gr[q] == gc) ? 1.0 : 0.0;
            }
            T[(int64_t)c * B + r] = v;
            ss += v * v;
        }
    }
    if (norm2) {
        __shared__ double red[4];
        double w = wave_sum(ss);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
        __syncthreads();
        if (threadIdx.x == 0) norm2[t] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

template <int B, int MODE>
__global__ __launch_bounds__(256) void gen_tiles_kernel(double *__restrict__ tiles,
                                                        const double *__restrict__ x,
                                                        const double *__restrict__ y, int64_t n,
                                                        gl_theta th, Geom geo, double *__restrict__ norm2)
{
    gen_tiles_body<B, MODE>(tiles, x, y, n, th, geo, norm2, blockIdx.x);
}

template <int B>
static void launch_gen_tiles_b(double *tiles, const double *x, const double *y, int64_t n, int64_t nt,
                               gl_theta th, Geom geo, double *norm2, hipStream_t s)
{
    dim3 grid((unsigned)tile_count(nt));
    if (geo.metric != GL_EUCLIDEAN)
        gen_tiles_kernel<B, GEN_ANY><<<grid, 256, 0, s>>>(tiles, x, y, n, th, geo, norm2);
    else if (matern_setup(th.theta1, th.theta2, th.theta3).kind != 0)
        gen_tiles_kernel<B, GEN_CLOSED><<<grid, 256, 0, s>>>(tiles, x, y, n, th, geo, norm2);
    else
        gen_tiles_kernel<B, GEN_EUCLID><<<grid, 256, 0, s>>>(tiles, x, y, n, th, geo, norm2);
}

void launch_gen_tiles(double *tiles, const double *x, const double *y, int64_t n, int b, int64_t nt,
                      gl_theta th, Geom geo, double *norm2, hipStream_t s)
{
    switch (b) {
    case 128: launch_gen_tiles_b<128>(tiles, x, y, n, nt, th, geo, norm2, s); break;
    case 256: launch_gen_tiles_b<256>(tiles, x, y, n, nt, th, geo, norm2, s); break;
    case 384: launch_gen_tiles_b<384>(tiles, x, y, n, nt, th, geo, norm2, s); break;
    default: launch_gen_tiles_b<512>(tiles, x, y, n, nt, th, geo, norm2, s); break;
    }
}

// The same, with θ read from device memory (replayed hipGraphs: the graph
// stays valid while θ changes between replays).
template <int B, int MODE>
__global__ __launch_bounds__(256) void gen_tiles_dev_kernel(double *__restrict__ tiles, const double *__restrict__ x,
                                                            const double *__restrict__ y, int64_t n,
                                                            const gl_theta *__restrict__ thp, Geom geo)
{
    gen_tiles_body<B, MODE>(tiles, x, y, n, *thp, geo, nullptr, blockIdx.x);
}

template <int B>
static void launch_gen_tiles_dev_b(double *tiles, const double *x, const double *y, int64_t n, int64_t nt,
                                   const gl_theta *thp, Geom geo, hipStream_t s)
{
    dim3 grid((unsigned)tile_count(nt));
    if (geo.metric == GL_EUCLIDEAN) gen_tiles_dev_kernel<B, GEN_EUCLID><<<grid, 256, 0, s>>>(tiles, x, y, n, thp, geo);
    else gen_tiles_dev_kernel<B, GEN_ANY><<<grid, 256, 0, s>>>(tiles, x, y, n, thp, geo);
}

void launch_gen_tiles_dev(double *tiles, const double *x, const double *y, int64_t n, int b, int64_t nt,
                          const gl_theta *thp, Geom geo, hipStream_t s)
{
    switch (b) {
    case 128: launch_gen_tiles_dev_b<128>(tiles, x, y, n, nt, thp, geo, s); break;
    case 256: launch_gen_tiles_dev_b<256>(tiles, x, y, n, nt, thp, geo, s); break;
    case 384: launch_gen_tiles_dev_b<384>(tiles, x, y, n, nt, thp, geo, s); break;
    default: launch_gen_tiles_dev_b<512>(tiles, x, y, n, nt, thp, geo, s); break;
    }
}

template <int B, int MODE>
__global__ __launch_bounds__(256) void gen_batched_kernel(const BatchReq *__restrict__ d, int count)
{
    const int64_t g = blockIdx.x;
    const int r = GL_BATCH_FIND(d, count, g, o_gen);
    const BatchReq &q = d[r];
    gen_tiles_body<B, MODE>(q.tiles, q.x, q.y, q.n, q.th, q.geo, nullptr, g - q.o_gen);
}

template <int B>
static void launch_gen_batched_b(const BatchReq *d, int count, int64_t tiles, bool euclid, hipStream_t s)
{
    if (euclid) gen_batched_kernel<B, GEN_EUCLID><<<(unsigned)tiles, 256, 0, s>>>(d, count);
    else gen_batched_kernel<B, GEN_ANY><<<(unsigned)tiles, 256, 0, s>>>(d, count);
}

void launch_gen_batched(int b, const BatchReq *d, int count, int64_t tiles, bool euclid, hipStream_t s)
{
    if (tiles <= 0) return;
    switch (b) {
    case 128: launch_gen_batched_b<128>(d, count, tiles, euclid, s); break;
    case 256: launch_gen_batched_b<256>(d, count, tiles, euclid, s); break;
    case 384: launch_gen_batched_b<384>(d, count, tiles, euclid, s); break;
    default: launch_gen_batched_b<512>(d, count, tiles, euclid, s); break;
    }
}

// Dense column-major n1×n2 covariance between two point sets: out[i + j*ld].
// Block: 256 rows × 16 columns.
__global__ __launch_bounds__(256) void gen_dense_kernel(const double *__restrict__ x1,
                                                        const double *__restrict__ y1, int64_t n1,
                                                        const double *__restrict__ x2,
                                                        const double *__restrict__ y2, int64_t n2,
                                                        gl_theta th, Geom geo, double *__restrict__ out,
                                                        int64_t ld)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * 16;
    const MaternSetup ms = matern_setup(th.theta1, th.theta2, th.theta3);
    __shared__ BesselTab tab;
    bessel_tab_init(ms, tab);
    if (i >= n1) return;
    const double xi = x1[i], yi = y1[i];
    for (int c = 0; c < 16; ++c) {
        int64_t j = j0 + c;
        if (j >= n2) break;
        out[i + j * ld] = matern_eval(ms, geo_dist(geo, xi, yi, x2[j], y2[j]), &tab);
    }
}

void launch_gen_dense(const double *x1, const double *y1, int64_t n1, const double *x2,
                      const double *y2, int64_t n2, gl_theta th, Geom geo, double *out, int64_t ld,
                      hipStream_t s)
{
    dim3 grid((unsigned)ceil_div(n1, 256), (unsigned)ceil_div(n2, 16));
    gen_dense_kernel<<<grid, 256, 0, s>>>(x1, y1, n1, x2, y2, n2, th, geo, out, ld);
}

// Kriging, Eq. (5): Z1_k = Σ_j C(||s_new,k - s_j||) v_j with v = Σ22⁻¹ Z2.
// Σ12 is generated on the fly.  Workgroup (k, chunk) sums the chunk's
// KRIGE_CHUNK observed points for new point k into part[k * nchunk + chunk].
constexpr int KRIGE_CHUNK = 4096;

__global__ __launch_bounds__(256) void krige_kernel(const double *__restrict__ x,
                                                    const double *__restrict__ y, int64_t n,
                                                    const double *__restrict__ v, gl_theta th, Geom geo,
                                                    const double *__restrict__ xn,
                                                    const double *__restrict__ yn,
                                                    double *__restrict__ part, int64_t nchunk)
{
    const int64_t k = blockIdx.x;
    const int64_t c = blockIdx.y;
    const MaternSetup ms = matern_setup(th.theta1, th.theta2, th.theta3);
    __shared__ BesselTab tab;
    bessel_tab_init(ms, tab);
    const double xk = xn[k], yk = yn[k];
    const int64_t j0 = c * KRIGE_CHUNK;
    const int64_t j1 = min(n, j0 + KRIGE_CHUNK);
    double acc = 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += 256)
        acc += matern_eval(ms, geo_dist(geo, xk, yk, x[j], y[j]), &tab) * v[j];
    __shared__ double red[4];
    double w = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) part[k * nchunk + c] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void krige_reduce_kernel(const double *__restrict__ part, int64_t m, int64_t nchunk,
                                    double *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= m) return;
    double s = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) s += part[k * nchunk + c];
    out[k] = s;
}

void launch_krige(const double *x, const double *y, int64_t n, const double *v, gl_theta th, Geom geo,
                  const double *xn, const double *yn, int64_t m, double *part, int64_t nchunk,
                  hipStream_t s)
{
    dim3 grid((unsigned)m, (unsigned)nchunk);
    krige_kernel<<<grid, 256, 0, s>>>(x, y, n, v, th, geo, xn, yn, part, nchunk);
}

void launch_krige_reduce(const double *part, int64_t m, int64_t nchunk, double *out, hipStream_t s)
{
    krige_reduce_kernel<<<(unsigned)ceil_div(m, 256), 256, 0, s>>>(part, m, nchunk, out);
}

int64_t krige_chunks(int64_t n) { return ceil_div(n, KRIGE_CHUNK); }

// Right-hand sides of the kriging variances (Eq. 4), transposed: tile (c, i)
// of st (b×b column-major) holds C(||s_new,r - s_p||) for new location
// c·b + r and observed location i·b + p; zero where either is padding.  One
// workgroup per tile; stores are coalesced along r.
template <int B>
__global__ __launch_bounds__(256) void gen_rhs_kernel(double *__restrict__ st, const double *__restrict__ x,
                                                      const double *__restrict__ y, int64_t n, int64_t nt,
                                                      const double *__restrict__ xn, const double *__restrict__ yn,
                                                      int64_t m, gl_theta th, Geom geo)
{
    const int64_t t = blockIdx.x;
    const int64_t c = t / nt, i = t % nt;
    const MaternSetup ms = matern_setup(th.theta1, th.theta2, th.theta3);
    __shared__ BesselTab tab;
    bessel_tab_init(ms, tab);
    double *T = st + t * (int64_t)B * B;
    constexpr int RPT = (B + 255) / 256;
    double xr[RPT], yr[RPT];
    bool rok[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = threadIdx.x + 256 * q;
        const int64_t kn = c * B + r;
        rok[q] = (r < B) && kn < m;
        xr[q] = rok[q] ? xn[kn] : 0.0;
        yr[q] = rok[q] ? yn[kn] : 0.0;
    }
    for (int p = 0; p < B; ++p) {
        const int64_t gp = i * B + p;
        const bool pok = gp < n;
        const double xp = pok ? x[gp] : 0.0;
        const double yp = pok ? y[gp] : 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = threadIdx.x + 256 * q;
            if (r >= B) continue;
            T[(int64_t)p * B + r] = (pok && rok[q]) ? matern_eval(ms, geo_dist(geo, xr[q], yr[q], xp, yp), &tab) : 0.0;
        }
    }
}

void launch_gen_rhs(double *st, const double *x, const double *y, int64_t n, int b, int64_t nt, const double *xn,
                    const double *yn, int64_t m, int64_t chunks, gl_theta th, Geom geo, hipStream_t s)
{
    const unsigned grid = (unsigned)(chunks * nt);
    switch (b) {
    case 128: gen_rhs_kernel<128><<<grid, 256, 0, s>>>(st, x, y, n, nt, xn, yn, m, th, geo); break;
    case 256: gen_rhs_kernel<256><<<grid, 256, 0, s>>>(st, x, y, n, nt, xn, yn, m, th, geo); break;
    case 384: gen_rhs_kernel<384><<<grid, 256, 0, s>>>(st, x, y, n, nt, xn, yn, m, th, geo); break;
    default: gen_rhs_kernel<512><<<grid, 256, 0, s>>>(st, x, y, n, nt, xn, yn, m, th, geo); break;
    }
}

}  // namespace gl
