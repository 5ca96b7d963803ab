// Panel triangular solve (the TRSM task of the tile algorithm, Sec. 5.2):
// L_ik = A_ik L_kk⁻ᵀ for every tile i > k of column k.
//
// Workgroup (i, strip) owns 64 rows of tile (i, k), the only writer of those
// rows, and solves them in place in 64-column blocks J, all on the matrix
// cores:
//   T      = A[:, J] - X[:, 0:J] · L_kk[J, 0:J]ᵀ
//   X[:, J] = T · D_J⁻ᵀ
// where D_J⁻¹ is the inverse of the J-th 64×64 diagonal block of L_kk, left in
// `dinv` by the POTRF of the same step.  The product streams 16-column chunks
// of X and L_kk through LDS, double-buffered; X[:, 0:J] was written by this
// workgroup in earlier blocks (visible after the block barrier).
#include "batch.hpp"
#include "common.hpp"
#include "mfma.hpp"

namespace gl {

constexpr int TB = 64;  // column block and strip height
constexpr int TC = 16;  // k chunk
constexpr int TP = TB + 16;  // LDS row pitch (bank spread of the 16-lane groups)

// Strip `strip` (64 rows) of X <- X L⁻ᵀ, X and L b×b column-major (ld b),
// dinv the inverses of L's 64×64 diagonal blocks.
template <int B>
__device__ __forceinline__ void trsm_core(const double *__restrict__ L, double *__restrict__ X,
                                          const double *__restrict__ dinv, int strip)
{
    const int r0 = strip * TB;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    // chunk buffers during the product (Xs[b][kc][r] = X[r0 + r][k0 + kc],
    // Ls[b][kc][j] = L[J + j][k0 + kc]); D_J⁻¹ reuses them afterwards
    __shared__ double buf[2 * TC * TP * 2];
    __shared__ double Tt[TB][TP];  // Tt[c][r] = T[r][c]
    auto Xs = reinterpret_cast<double(*)[TC][TP]>(buf);
    auto Ls = reinterpret_cast<double(*)[TC][TP]>(buf + 2 * TC * TP);
    double *Di = buf;  // Di[c * TP + r] = (D_J⁻¹)[r][c]

    const int lkc = tid >> 4, lr = (tid & 15) * 4;  // loader: column lkc, rows lr..lr+3

    for (int J = 0; J < B; J += TB) {
        const int nch = J / TC;
        d4 acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = (d4){0.0, 0.0, 0.0, 0.0};
        d2 rx[2], rl[2];
        if (nch > 0) {
            const d2 *px = reinterpret_cast<const d2 *>(X + (int64_t)lkc * B + r0 + lr);
            const d2 *pl = reinterpret_cast<const d2 *>(L + (int64_t)lkc * B + J + lr);
            rx[0] = px[0];
            rx[1] = px[1];
            rl[0] = pl[0];
            rl[1] = pl[1];
            *reinterpret_cast<d2 *>(&Xs[0][lkc][lr]) = rx[0];
            *reinterpret_cast<d2 *>(&Xs[0][lkc][lr + 2]) = rx[1];
            *reinterpret_cast<d2 *>(&Ls[0][lkc][lr]) = rl[0];
            *reinterpret_cast<d2 *>(&Ls[0][lkc][lr + 2]) = rl[1];
        }
        __syncthreads();
        for (int ch = 0; ch < nch; ++ch) {
            const int cur = ch & 1;
            if (ch + 1 < nch) {
                const int64_t col = (int64_t)(ch + 1) * TC + lkc;
                const d2 *px = reinterpret_cast<const d2 *>(X + col * B + r0 + lr);
                const d2 *pl = reinterpret_cast<const d2 *>(L + col * B + J + lr);
                rx[0] = px[0];
                rx[1] = px[1];
                rl[0] = pl[0];
                rl[1] = pl[1];
            }
            // wave w: columns w*16.. of the block; four 16-row groups of the strip
#pragma unroll
            for (int kk = 0; kk < TC; kk += 4) {
                const double xl = Ls[cur][kk + (lane >> 4)][wave * 16 + (lane & 15)];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
                    acc[rb] = mfma_f64(xl, Xs[cur][kk + (lane >> 4)][rb * 16 + (lane & 15)], acc[rb]);
            }
            if (ch + 1 < nch) {
                *reinterpret_cast<d2 *>(&Xs[cur ^ 1][lkc][lr]) = rx[0];
                *reinterpret_cast<d2 *>(&Xs[cur ^ 1][lkc][lr + 2]) = rx[1];
                *reinterpret_cast<d2 *>(&Ls[cur ^ 1][lkc][lr]) = rl[0];
                *reinterpret_cast<d2 *>(&Ls[cur ^ 1][lkc][lr + 2]) = rl[1];
            }
            __syncthreads();
        }
        // T = A[:, J] - product (result row q of lane l: block column w*16 + l/16 + 4q,
        // lane % 16: strip row), and D_J⁻¹ into LDS
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = wave * 16 + mfma_row(lane, q);
                const int r = rb * 16 + mfma_col(lane);
                Tt[c][r] = X[(int64_t)(J + c) * B + r0 + r] - acc[rb][q];
            }
        const double *dv = dinv + (int64_t)(J / TB) * TB * TB;
        for (int e = tid; e < TB * TB; e += 256) Di[(e >> 6) * TP + (e & 63)] = dv[e];
        __syncthreads();
        // X[:, J] = T · D_J⁻ᵀ: X[r][c] = Σ_m T[r][m] D⁻¹[c][m]
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < TB; kk += 4) {
            const int m = kk + (lane >> 4);
            const double xd = Di[m * TP + wave * 16 + (lane & 15)];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) acc[rb] = mfma_f64(xd, Tt[m][rb * 16 + (lane & 15)], acc[rb]);
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = wave * 16 + mfma_row(lane, q);
                const int r = rb * 16 + mfma_col(lane);
                X[(int64_t)(J + c) * B + r0 + r] = acc[rb][q];
            }
        __syncthreads();
    }
}

// Strip `strip` of panel tile i = k + 1 + tix.
template <int B>
__device__ __forceinline__ void trsm_body(double *__restrict__ tiles, int64_t k,
                                          const double *__restrict__ dinv,
                                          const int64_t *__restrict__ info, int64_t tix, int strip)
{
    if (*info != 0) return;
    __builtin_amdgcn_s_setprio(3);  // critical path of the step schedule
    trsm_core<B>(tiles + tile_offset(k, k, B), tiles + tile_offset(k + 1 + tix, k, B), dinv, strip);
}

template <int B>
__global__ __launch_bounds__(256) void trsm_kernel(double *__restrict__ tiles, int64_t k,
                                                   const double *__restrict__ dinv,
                                                   const int64_t *__restrict__ info)
{
    trsm_body<B>(tiles, k, dinv, info, blockIdx.x, blockIdx.y);
}

void launch_trsm(double *tiles, int b, int64_t nt, int64_t k, const double *dinv, const int64_t *info,
                 hipStream_t s)
{
    const int64_t m = nt - k - 1;
    if (m <= 0) return;
    dim3 grid((unsigned)m, (unsigned)(b / TB));
    switch (b) {
    case 128: trsm_kernel<128><<<grid, 256, 0, s>>>(tiles, k, dinv, info); break;
    case 256: trsm_kernel<256><<<grid, 256, 0, s>>>(tiles, k, dinv, info); break;
    case 384: trsm_kernel<384><<<grid, 256, 0, s>>>(tiles, k, dinv, info); break;
    default: trsm_kernel<512><<<grid, 256, 0, s>>>(tiles, k, dinv, info); break;
    }
}

template <int B>
__global__ __launch_bounds__(256) void trsm_batched_kernel(const BatchReq *__restrict__ d, int count)
{
    const int64_t g = blockIdx.x;
    const int r = GL_BATCH_FIND(d, count, g, o_trsm);
    const BatchReq &q = d[r];
    const int64_t local = g - q.o_trsm;
    trsm_body<B>(q.tiles, q.k, q.dinv, q.info, local / (B / TB), (int)(local % (B / TB)));
}

void launch_trsm_batched(int b, const BatchReq *d, int count, int64_t blocks, hipStream_t s)
{
    if (blocks <= 0) return;
    switch (b) {
    case 128: trsm_batched_kernel<128><<<(unsigned)blocks, 256, 0, s>>>(d, count); break;
    case 256: trsm_batched_kernel<256><<<(unsigned)blocks, 256, 0, s>>>(d, count); break;
    case 384: trsm_batched_kernel<384><<<(unsigned)blocks, 256, 0, s>>>(d, count); break;
    default: trsm_batched_kernel<512><<<(unsigned)blocks, 256, 0, s>>>(d, count); break;
    }
}

// Many right-hand sides (kriging variances, Eq. 4): U = L⁻¹ S is solved in
// the transposed form Uᵀ L_kkᵀ = Sᵀ, the panel form above.  st holds chunks
// of b right-hand sides as nt tiles each (tile (c, i): b×b column-major, row
// = right-hand side, column = location of tile i).  Diagonal step k solves
// tile (c, k) of every chunk c.
template <int B>
__global__ __launch_bounds__(256) void mrhs_diag_kernel(const double *__restrict__ tiles, double *__restrict__ st,
                                                        int64_t nt, int64_t k, const double *__restrict__ dinv)
{
    trsm_core<B>(tiles + tile_offset(k, k, B), st + ((int64_t)blockIdx.x * nt + k) * B * B, dinv, blockIdx.y);
}

void launch_mrhs_diag(const double *tiles, double *st, int b, int64_t nt, int64_t k, const double *dinv,
                      int64_t chunks, hipStream_t s)
{
    dim3 grid((unsigned)chunks, (unsigned)(b / TB));
    switch (b) {
    case 128: mrhs_diag_kernel<128><<<grid, 256, 0, s>>>(tiles, st, nt, k, dinv); break;
    case 256: mrhs_diag_kernel<256><<<grid, 256, 0, s>>>(tiles, st, nt, k, dinv); break;
    case 384: mrhs_diag_kernel<384><<<grid, 256, 0, s>>>(tiles, st, nt, k, dinv); break;
    default: mrhs_diag_kernel<512><<<grid, 256, 0, s>>>(tiles, st, nt, k, dinv); break;
    }
}

}  // namespace gl
