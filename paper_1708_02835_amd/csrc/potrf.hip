// Diagonal-tile Cholesky factorisation (the POTRF task of the tile algorithm,
// Sec. 4.2 and Alg. 2 step 3).
//
// One workgroup of 256 threads factors the b×b tile A_kk = L_kk L_kkᵀ in place
// (lower triangle), blocked right-looking with a 32-column panel:
//   1. the panel (rows s..b-1, columns s..s+31) is held in registers, two rows
//      per thread at most, and factored column by column; the pivot row's
//      entries are exchanged through LDS;
//   2. the trailing lower triangle A[s+32:, s+32:] -= P Pᵀ is updated with the
//      FP64 16x16x4 matrix-core product, the four waves sharing the 16×16
//      blocks of the lower triangle.
// A non-positive (or NaN) pivot stores the 1-based global column in *info and
// stops; every later kernel of the factorisation then returns immediately.
// The tile's contribution 2 Σ log L_rr over rows r < n goes to logsum[k].
#include "common.hpp"
#include "mfma.hpp"

namespace gl {

constexpr int PNB = 32;  // panel width

template <int B>
__global__ __launch_bounds__(256) void potrf_kernel(double *__restrict__ tiles, int64_t k, int64_t n,
                                                    int64_t *__restrict__ info,
                                                    double *__restrict__ logsum)
{
    if (*info != 0) return;
    double *A = tiles + tile_offset(k, k, B);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    constexpr int RPT = (B + 255) / 256;
    __shared__ double pcol[PNB];
    __shared__ double red[4];

    for (int s = 0; s < B; s += PNB) {
        double p[RPT][PNB];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = s + tid + 256 * q;
#pragma unroll
            for (int c = 0; c < PNB; ++c) p[q][c] = (row < B) ? A[(int64_t)(s + c) * B + row] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < PNB; ++c) {
            // rows s+c .. s+PNB-1 of column c are owned by threads c .. PNB-1 (q = 0)
            if (tid >= c && tid < PNB) pcol[tid] = p[0][c];
            __syncthreads();
            const double piv = pcol[c];
            if (!(piv > 0.0)) {
                if (tid == 0) *info = k * B + s + c + 1;
                return;  // uniform: every thread read the same pivot
            }
            const double d = sqrt(piv);
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int row = s + tid + 256 * q;
                if (row == s + c) p[q][c] = d;
                else if (row > s + c) p[q][c] = p[q][c] / d;
            }
#pragma unroll
            for (int j = c + 1; j < PNB; ++j) {
                const double ljc = pcol[j] / d;
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int row = s + tid + 256 * q;
                    if (row >= s + j) p[q][j] -= p[q][c] * ljc;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = s + tid + 256 * q;
            if (row < B) {
#pragma unroll
                for (int c = 0; c < PNB; ++c)
                    if (row >= s + c) A[(int64_t)(s + c) * B + row] = p[q][c];
            }
        }
        __syncthreads();

        // trailing update of the lower triangle below/right of the panel
        const int R = B - s - PNB;
        if (R > 0) {
            const int nb = R / 16;
            const int nblk = nb * (nb + 1) / 2;
            const int r0 = s + PNB;
            for (int blk = wave; blk < nblk; blk += 4) {
                int bi = (int)((sqrt(8.0 * blk + 1.0) - 1.0) * 0.5);
                while (bi * (bi + 1) / 2 > blk) --bi;
                while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
                const int bj = blk - bi * (bi + 1) / 2;
                d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < PNB; kk += 4) {
                    const int64_t col = s + kk + (lane >> 4);
                    const double a = A[col * B + r0 + bi * 16 + (lane & 15)];
                    const double b = A[col * B + r0 + bj * 16 + (lane & 15)];
                    acc = mfma_f64(a, b, acc);
                }
                const int64_t ccol = r0 + bj * 16 + mfma_col(lane);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rrow = r0 + bi * 16 + mfma_row(lane, r);
                    A[ccol * B + rrow] -= acc[r];
                }
            }
        }
        __syncthreads();
    }

    // 2 Σ log L_rr over the rows that are not padding
    double acc = 0.0;
    for (int r = tid; r < B; r += 256)
        if (k * B + r < n) acc += log(A[(int64_t)r * B + r]);
    double w = wave_sum(acc);
    if (lane == 0) red[wave] = w;
    __syncthreads();
    if (tid == 0) logsum[k] = 2.0 * ((red[0] + red[1]) + (red[2] + red[3]));
}

void launch_potrf(double *tiles, int b, int64_t k, int64_t n, int64_t *info, double *logsum,
                  hipStream_t s)
{
    switch (b) {
    case 128: potrf_kernel<128><<<1, 256, 0, s>>>(tiles, k, n, info, logsum); break;
    case 256: potrf_kernel<256><<<1, 256, 0, s>>>(tiles, k, n, info, logsum); break;
    case 384: potrf_kernel<384><<<1, 256, 0, s>>>(tiles, k, n, info, logsum); break;
    default: potrf_kernel<512><<<1, 256, 0, s>>>(tiles, k, n, info, logsum); break;
    }
}

}  // namespace gl
