// Triangular solves, TRMV and the scalar reductions on the packed tile factor.
//
//  * forward solve w = L⁻¹ Z (Alg. 2 step 4, "dtrsm" with one right-hand side),
//    by tile columns: solve the diagonal block, then subtract L_ik w_k from the
//    blocks below; the diagonal-block kernel also emits the tile's part of
//    wᵀw (Alg. 2 step 6);
//  * backward solve X = L⁻ᵀ w (the second half of "dposv" in Alg. 3);
//  * Z = L e (Alg. 1 step 7, "dtrmm");
//  * the final fixed-order reduction of the per-tile log-det and quadratic
//    form parts into l(θ) (Alg. 2 step 7, Eq. (1)).
// Every reduction has a fixed order, so results do not depend on scheduling.
#include <math.h>

#include "batch.hpp"
#include "common.hpp"
#include "mfma.hpp"

namespace gl {

// v_k <- L_kk⁻¹ v_k by 64-row blocks J, using the inverted diagonal blocks
// D_J⁻¹ that POTRF left in `dinv`:  t = v_J - L[J, 0:J] w[0:J],  w_J = D_J⁻¹ t.
// Both products are split over four thread groups with fixed-order partial
// sums.  The tile's part of wᵀw (rows < n) goes to quad_part[k].
template <int B>
__device__ __forceinline__ void fwd_diag_body(const double *__restrict__ tiles, int64_t k, int64_t n,
                                              double *__restrict__ v, double *__restrict__ quad_part,
                                              const double *__restrict__ dinv,
                                              const int64_t *__restrict__ info)
{
    if (info && *info != 0) return;
    __builtin_amdgcn_s_setprio(3);  // critical path of the step schedule
    const double *L = tiles + tile_offset(k, k, B);
    double *vk = v + k * B;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int r = tid & 63, g = tid >> 6;
    __shared__ double xs[B];
    __shared__ double t[64];
    __shared__ double part[4][64];
    __shared__ double red[4];
    for (int q = tid; q < B; q += 256) xs[q] = vk[q];
    __syncthreads();
    for (int J = 0; J < B; J += 64) {
        double acc = 0.0;
        for (int c = g; c < J; c += 4) acc += L[(int64_t)c * B + J + r] * xs[c];
        part[g][r] = acc;
        __syncthreads();
        if (tid < 64) t[r] = xs[J + r] - ((part[0][r] + part[1][r]) + (part[2][r] + part[3][r]));
        __syncthreads();
        const double *dv = dinv + (int64_t)(J / 64) * 64 * 64;
        acc = 0.0;
        for (int m = g; m < 64; m += 4) acc += dv[m * 64 + r] * t[m];
        part[g][r] = acc;
        __syncthreads();
        if (tid < 64) xs[J + r] = (part[0][r] + part[1][r]) + (part[2][r] + part[3][r]);
        __syncthreads();
    }
    double q = 0.0;
    for (int rr = tid; rr < B; rr += 256) {
        vk[rr] = xs[rr];
        if (k * B + rr < n) q += xs[rr] * xs[rr];
    }
    if (quad_part) {
        double w = wave_sum(q);
        if (lane == 0) red[wave] = w;
        __syncthreads();
        if (tid == 0) quad_part[k] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

template <int B>
__global__ __launch_bounds__(256) void fwd_diag_kernel(const double *__restrict__ tiles, int64_t k,
                                                       int64_t n, double *__restrict__ v,
                                                       double *__restrict__ quad_part,
                                                       const double *__restrict__ dinv,
                                                       const int64_t *__restrict__ info)
{
    fwd_diag_body<B>(tiles, k, n, v, quad_part, dinv, info);
}

// v_i -= L_ik v_k for every tile i > k; workgroup (tile i = k + 1 + tix, 64-row strip).
template <int B>
__device__ __forceinline__ void fwd_update_body(const double *__restrict__ tiles, int64_t k,
                                                double *__restrict__ v, const int64_t *__restrict__ info,
                                                int64_t tix, int strip)
{
    if (info && *info != 0) return;
    __builtin_amdgcn_s_setprio(3);
    const int64_t i = k + 1 + tix;
    const int r0 = strip * 64;
    const double *L = tiles + tile_offset(i, k, B);
    const int tid = threadIdx.x;
    __shared__ double wk[B];
    __shared__ double red[4][64];
    for (int c = tid; c < B; c += 256) wk[c] = v[k * B + c];
    __syncthreads();
    const int r = tid & 63, g = tid >> 6;
    double acc = 0.0;
    for (int c = g; c < B; c += 4) acc += L[(int64_t)c * B + r0 + r] * wk[c];
    red[g][r] = acc;
    __syncthreads();
    if (g == 0) v[i * B + r0 + r] -= (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
}

template <int B>
__global__ __launch_bounds__(256) void fwd_update_kernel(const double *__restrict__ tiles, int64_t k,
                                                         double *__restrict__ v,
                                                         const int64_t *__restrict__ info)
{
    fwd_update_body<B>(tiles, k, v, info, blockIdx.x, blockIdx.y);
}

// v_k <- L_kk⁻ᵀ v_k, 64-row blocks from the bottom: the block's rows first
// receive the contributions of the solved rows below it (column dot products),
// then wave 0 back-substitutes the 64×64 block held in LDS.
template <int B>
__global__ __launch_bounds__(256) void bwd_diag_kernel(const double *__restrict__ tiles, int64_t k,
                                                       double *__restrict__ v)
{
    const double *L = tiles + tile_offset(k, k, B);
    double *vk = v + k * B;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    __shared__ double xs[B];
    __shared__ double Lb[64][65];  // Lb[c][r] = L[s + r][s + c]
    for (int r = tid; r < B; r += 256) xs[r] = vk[r];
    __syncthreads();
    for (int s = B - 64; s >= 0; s -= 64) {
        // xs[c] -= Σ_{r >= s+64} L[r][c] xs[r] for the 64 columns c of this block
        for (int cc = wave * 16; cc < wave * 16 + 16; ++cc) {
            const int c = s + cc;
            double acc = 0.0;
            for (int r = s + 64 + lane; r < B; r += 64) acc += L[(int64_t)c * B + r] * xs[r];
            acc = wave_sum(acc);
            if (lane == 0) xs[c] -= acc;
        }
        for (int e = tid; e < 64 * 64; e += 256) {
            const int c = e >> 6, r = e & 63;
            Lb[c][r] = L[(int64_t)(s + c) * B + s + r];
        }
        __syncthreads();
        if (wave == 0) {
            double z = xs[s + lane];
            for (int c = 63; c >= 0; --c) {
                const double xc = __shfl(z, c, 64) / Lb[c][c];
                if (lane == c) z = xc;
                else if (lane < c) z -= Lb[lane][c] * xc;  // L[s + c][s + lane]
            }
            xs[s + lane] = z;
        }
        __syncthreads();
    }
    for (int r = tid; r < B; r += 256) vk[r] = xs[r];
}

// v_j -= L_kjᵀ v_k for every tile j < k; workgroup (j, 64-column strip),
// each wave 16 columns, one column dot product at a time.
template <int B>
__global__ __launch_bounds__(256) void bwd_update_kernel(const double *__restrict__ tiles, int64_t k,
                                                         double *__restrict__ v)
{
    const int64_t j = blockIdx.x;
    const int c0 = blockIdx.y * 64;
    const double *L = tiles + tile_offset(k, j, B);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    __shared__ double xk[B];
    for (int r = tid; r < B; r += 256) xk[r] = v[k * B + r];
    __syncthreads();
    for (int cc = wave * 16; cc < wave * 16 + 16; ++cc) {
        const int c = c0 + cc;
        double acc = 0.0;
        for (int r = lane; r < B; r += 64) acc += L[(int64_t)c * B + r] * xk[r];
        acc = wave_sum(acc);
        if (lane == 0) v[j * B + c] -= acc;
    }
}

// z_i = Σ_{j<i} L_ij e_j + tril(L_ii) e_i; workgroup (i, 64-row strip).
template <int B>
__global__ __launch_bounds__(256) void trmv_kernel(const double *__restrict__ tiles,
                                                   const double *__restrict__ e,
                                                   double *__restrict__ z)
{
    const int64_t i = blockIdx.x;
    const int r0 = blockIdx.y * 64;
    const int tid = threadIdx.x;
    const int r = tid & 63, g = tid >> 6;
    __shared__ double red[4][64];
    double acc = 0.0;
    for (int64_t j = 0; j <= i; ++j) {
        const double *L = tiles + tile_offset(i, j, B);
        const double *ej = e + j * B;
        const int cend = (j == i) ? (r0 + r + 1) : B;
        for (int c = g; c < cend; c += 4) acc += L[(int64_t)c * B + r0 + r] * ej[c];
    }
    red[g][r] = acc;
    __syncthreads();
    if (g == 0) z[i * B + r0 + r] = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
}

// One wave: logdet = Σ_k logsum[k], quad = Σ_k quad_part[k], l by Eq. (1).
__device__ __forceinline__ void final_reduce_body(const double *__restrict__ logsum,
                                                  const double *__restrict__ quad_part, int64_t nt,
                                                  int64_t n, const int64_t *__restrict__ info,
                                                  DevResult *__restrict__ res)
{
    const int lane = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t t = lane; t < nt; t += 64) {
        a += logsum[t];
        b += quad_part[t];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
        const int64_t inf = *info;
        res->info = inf;
        if (inf != 0) {
            res->loglik = -INFINITY;
            res->logdet = NAN;
            res->quad = NAN;
        } else {
            res->logdet = a;
            res->quad = b;
            res->loglik = -0.5 * b - 0.5 * a - 0.5 * (double)n * log(2.0 * M_PI);
        }
    }
}

__global__ void final_reduce_kernel(const double *__restrict__ logsum,
                                    const double *__restrict__ quad_part, int64_t nt, int64_t n,
                                    const int64_t *__restrict__ info, DevResult *__restrict__ res)
{
    final_reduce_body(logsum, quad_part, nt, n, info, res);
}

__global__ void fill_kernel(double *__restrict__ p, int64_t count, double v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void copy_pad_kernel(const double *__restrict__ src, int64_t n, double *__restrict__ dst,
                                int64_t npad, double padv)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < npad) dst[i] = (i < n) ? src[i] : padv;
}

// Dense column-major copy of the n×n lower factor, zero strict upper triangle.
__global__ void tiles_to_dense_kernel(const double *__restrict__ tiles, int b, int64_t n,
                                      double *__restrict__ out, int64_t ld)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    for (int64_t c = blockIdx.y; c < n; c += gridDim.y) {
        double v = 0.0;
        if (r >= c) {
            const int64_t ti = r / b, tj = c / b;
            v = tiles[tile_offset(ti, tj, b) + (c % b) * b + (r % b)];
        }
        out[r + c * ld] = v;
    }
}

template <int B>
__global__ __launch_bounds__(256) void fwd_diag_batched_kernel(const BatchReq *__restrict__ d)
{
    const BatchReq &r = d[blockIdx.x];
    fwd_diag_body<B>(r.tiles, r.k, r.n, r.v, r.quad, r.dinv, r.info);
}

template <int B>
__global__ __launch_bounds__(256) void fwd_update_batched_kernel(const BatchReq *__restrict__ d, int count)
{
    const int64_t g = blockIdx.x;
    const int r = GL_BATCH_FIND(d, count, g, o_trsm);
    const BatchReq &q = d[r];
    const int64_t local = g - q.o_trsm;
    fwd_update_body<B>(q.tiles, q.k, q.v, q.info, local / (B / 64), (int)(local % (B / 64)));
}

__global__ void final_batched_kernel(const BatchReq *__restrict__ d)
{
    const BatchReq &r = d[blockIdx.x];
    if (!r.finishing) return;
    final_reduce_body(r.logsum, r.quad, r.nt, r.n, r.info, r.res);
}

// Padded copies of new requests' inputs, and their info word cleared.
__global__ void stage_batched_kernel(const BatchReq *__restrict__ d, int count)
{
    const int64_t g = blockIdx.x;
    const int r = GL_BATCH_FIND(d, count, g, o_stage);
    const BatchReq &q = d[r];
    const int64_t i = (g - q.o_stage) * 256 + threadIdx.x;
    if (i == 0) *q.info = 0;
    if (i >= q.npad) return;
    const bool in = i < q.n;
    q.x[i] = in ? q.sx[i] : 0.0;
    q.y[i] = in ? q.sy[i] : 0.0;
    q.v[i] = in ? q.sz[i] : 0.0;
}

void launch_fwd_diag_batched(int b, const BatchReq *d, int count, hipStream_t s)
{
    switch (b) {
    case 128: fwd_diag_batched_kernel<128><<<count, 256, 0, s>>>(d); break;
    case 256: fwd_diag_batched_kernel<256><<<count, 256, 0, s>>>(d); break;
    case 384: fwd_diag_batched_kernel<384><<<count, 256, 0, s>>>(d); break;
    default: fwd_diag_batched_kernel<512><<<count, 256, 0, s>>>(d); break;
    }
}

void launch_fwd_update_batched(int b, const BatchReq *d, int count, int64_t blocks, hipStream_t s)
{
    if (blocks <= 0) return;
    switch (b) {
    case 128: fwd_update_batched_kernel<128><<<(unsigned)blocks, 256, 0, s>>>(d, count); break;
    case 256: fwd_update_batched_kernel<256><<<(unsigned)blocks, 256, 0, s>>>(d, count); break;
    case 384: fwd_update_batched_kernel<384><<<(unsigned)blocks, 256, 0, s>>>(d, count); break;
    default: fwd_update_batched_kernel<512><<<(unsigned)blocks, 256, 0, s>>>(d, count); break;
    }
}

void launch_final_batched(const BatchReq *d, int count, hipStream_t s)
{
    final_batched_kernel<<<count, 64, 0, s>>>(d);
}

void launch_stage_batched(const BatchReq *d, int count, int64_t blocks, hipStream_t s)
{
    if (blocks <= 0) return;
    stage_batched_kernel<<<(unsigned)blocks, 256, 0, s>>>(d, count);
}

#define GL_DISPATCH_B(b, KERNEL, GRID, ...)                                   \
    switch (b) {                                                              \
    case 128: KERNEL<128><<<GRID, 256, 0, s>>>(__VA_ARGS__); break;           \
    case 256: KERNEL<256><<<GRID, 256, 0, s>>>(__VA_ARGS__); break;           \
    case 384: KERNEL<384><<<GRID, 256, 0, s>>>(__VA_ARGS__); break;           \
    default: KERNEL<512><<<GRID, 256, 0, s>>>(__VA_ARGS__); break;            \
    }

void launch_fwd_diag(const double *tiles, int b, int64_t k, int64_t n, double *v, double *quad_part,
                     const double *dinv, const int64_t *info, hipStream_t s)
{
    GL_DISPATCH_B(b, fwd_diag_kernel, dim3(1), tiles, k, n, v, quad_part, dinv, info);
}

void launch_fwd_update(const double *tiles, int b, int64_t nt, int64_t k, double *v,
                       const int64_t *info, hipStream_t s)
{
    if (nt - k - 1 <= 0) return;
    dim3 grid((unsigned)(nt - k - 1), (unsigned)(b / 64));
    GL_DISPATCH_B(b, fwd_update_kernel, grid, tiles, k, v, info);
}

void launch_bwd_diag(const double *tiles, int b, int64_t k, double *v, hipStream_t s)
{
    GL_DISPATCH_B(b, bwd_diag_kernel, dim3(1), tiles, k, v);
}

void launch_bwd_update(const double *tiles, int b, int64_t k, double *v, hipStream_t s)
{
    if (k <= 0) return;
    dim3 grid((unsigned)k, (unsigned)(b / 64));
    GL_DISPATCH_B(b, bwd_update_kernel, grid, tiles, k, v);
}

void launch_trmv(const double *tiles, int b, int64_t nt, const double *e, double *z, hipStream_t s)
{
    dim3 grid((unsigned)nt, (unsigned)(b / 64));
    GL_DISPATCH_B(b, trmv_kernel, grid, tiles, e, z);
}

void launch_final_reduce(const double *logsum, const double *quad_part, int64_t nt, int64_t n,
                         const int64_t *info, DevResult *res, hipStream_t s)
{
    final_reduce_kernel<<<1, 64, 0, s>>>(logsum, quad_part, nt, n, info, res);
}

void launch_fill(double *p, int64_t count, double v, hipStream_t s)
{
    if (count <= 0) return;
    fill_kernel<<<(unsigned)ceil_div(count, 256), 256, 0, s>>>(p, count, v);
}

void launch_copy_pad(const double *src, int64_t n, double *dst, int64_t npad, double padv,
                     hipStream_t s)
{
    copy_pad_kernel<<<(unsigned)ceil_div(npad, 256), 256, 0, s>>>(src, n, dst, npad, padv);
}

void launch_tiles_to_dense(const double *tiles, int b, int64_t n, double *out, int64_t ld,
                           hipStream_t s)
{
    dim3 grid((unsigned)ceil_div(n, 256), (unsigned)(n < 65535 ? n : 65535));
    tiles_to_dense_kernel<<<grid, 256, 0, s>>>(tiles, b, n, out, ld);
}

// Kriging variances from the solved right-hand sides U (layout of st):
// part[(c·nt + i)·b + r] = Σ_p U(c, i)[r, p]² per tile (one workgroup per
// tile, threads along r), then var[c·b + r] = θ1 - Σ_i part[...] in tile
// order (fixed order, deterministic).
template <int B>
__global__ __launch_bounds__(256) void rhs_sq_partial_kernel(const double *__restrict__ st, double *__restrict__ part)
{
    const int64_t t = blockIdx.x;
    const double *T = st + t * (int64_t)B * B;
    for (int r = threadIdx.x; r < B; r += 256) {
        double acc = 0.0;
        for (int p = 0; p < B; ++p) {
            const double u = T[(int64_t)p * B + r];
            acc += u * u;
        }
        part[t * B + r] = acc;
    }
}

__global__ void rhs_var_kernel(const double *__restrict__ part, int64_t nt, int b, int64_t m, double theta1,
                               double *__restrict__ var)
{
    const int64_t kn = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (kn >= m) return;
    const int64_t c = kn / b, r = kn % b;
    double acc = 0.0;
    for (int64_t i = 0; i < nt; ++i) acc += part[(c * nt + i) * b + r];
    var[kn] = theta1 - acc;
}

void launch_rhs_variance(const double *st, int b, int64_t nt, int64_t chunks, int64_t m, double theta1,
                         double *part, double *var, hipStream_t s)
{
    const unsigned grid = (unsigned)(chunks * nt);
    switch (b) {
    case 128: rhs_sq_partial_kernel<128><<<grid, 256, 0, s>>>(st, part); break;
    case 256: rhs_sq_partial_kernel<256><<<grid, 256, 0, s>>>(st, part); break;
    case 384: rhs_sq_partial_kernel<384><<<grid, 256, 0, s>>>(st, part); break;
    default: rhs_sq_partial_kernel<512><<<grid, 256, 0, s>>>(st, part); break;
    }
    rhs_var_kernel<<<(unsigned)ceil_div(m, 256), 256, 0, s>>>(part, nt, b, m, theta1, var);
}

// Cross-validation helpers: gather three arrays through an index list, and
// the mean squared difference of two vectors (one workgroup, fixed order).
__global__ void gather3_kernel(const double *__restrict__ a, const double *__restrict__ b,
                               const double *__restrict__ c, const int64_t *__restrict__ idx, int64_t m,
                               double *__restrict__ oa, double *__restrict__ ob, double *__restrict__ oc)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int64_t j = idx[i];
    oa[i] = a[j];
    ob[i] = b[j];
    oc[i] = c[j];
}

void launch_gather3(const double *a, const double *b, const double *c, const int64_t *idx, int64_t m, double *oa,
                    double *ob, double *oc, hipStream_t s)
{
    gather3_kernel<<<(unsigned)ceil_div(m, 256), 256, 0, s>>>(a, b, c, idx, m, oa, ob, oc);
}

// out[idx[i]] = a[i]: the fold's predictions back to the input positions.
__global__ void scatter_kernel(const double *__restrict__ a, const int64_t *__restrict__ idx, int64_t m,
                               double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    out[idx[i]] = a[i];
}

void launch_scatter(const double *a, const int64_t *idx, int64_t m, double *out, hipStream_t s)
{
    scatter_kernel<<<(unsigned)ceil_div(m, 256), 256, 0, s>>>(a, idx, m, out);
}

__global__ __launch_bounds__(256) void mse_kernel(const double *__restrict__ p, const double *__restrict__ q,
                                                  int64_t m, double *__restrict__ out)
{
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 256) {
        const double d = p[i] - q[i];
        acc += d * d;
    }
    __shared__ double red[4];
    const double w = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) *out = ((red[0] + red[1]) + (red[2] + red[3])) / (double)m;
}

void launch_mse(const double *p, const double *q, int64_t m, double *out, hipStream_t s)
{
    mse_kernel<<<1, 256, 0, s>>>(p, q, m, out);
}

}  // namespace gl
