// Panel triangular solve (the TRSM task of the tile algorithm, Sec. 4.2):
// L_ik = A_ik L_kk⁻ᵀ for every tile i > k of column k.
//
// Workgroup (i, strip) owns 64 rows of tile (i, k), so it is the only writer
// of those rows and solves them in place.  The strip X (64 × b) is computed in
// 32-column blocks J:
//   T = A[:, J] - X[:, 0:J] · L_kk[J, 0:J]ᵀ        (FP64 matrix-core product)
//   X[:, J] = T · L_kk[J, J]⁻ᵀ                      (forward substitution per row)
// Columns 0:J of the strip were written by this workgroup in earlier blocks.
#include "common.hpp"
#include "mfma.hpp"

namespace gl {

constexpr int TNB = 32;  // column block
constexpr int TSH = 64;  // strip height

template <int B>
__global__ __launch_bounds__(256) void trsm_kernel(double *__restrict__ tiles, int64_t k,
                                                   const int64_t *__restrict__ info)
{
    if (*info != 0) return;
    const int64_t i = k + 1 + blockIdx.x;
    const int r0 = blockIdx.y * TSH;
    const double *L = tiles + tile_offset(k, k, B);
    double *X = tiles + tile_offset(i, k, B);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    __shared__ double T[TSH][TNB + 1];
    __shared__ double Ld[TNB][TNB + 1];

    for (int J = 0; J < B; J += TNB) {
        // wave w owns rows r0 + 16w .. +15 of the strip, two 16-column halves
        d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        for (int kk = 0; kk < J; kk += 4) {
            const int64_t col = kk + (lane >> 4);
            const double a = X[col * B + r0 + wave * 16 + (lane & 15)];
            const double b0 = L[col * B + J + (lane & 15)];
            const double b1 = L[col * B + J + 16 + (lane & 15)];
            acc0 = mfma_f64(a, b0, acc0);
            acc1 = mfma_f64(a, b1, acc1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + mfma_row(lane, r);
            const int c0 = mfma_col(lane);
            T[row][c0] = X[(int64_t)(J + c0) * B + r0 + row] - acc0[r];
            T[row][16 + c0] = X[(int64_t)(J + 16 + c0) * B + r0 + row] - acc1[r];
        }
        for (int e = tid; e < TNB * TNB; e += 256) {
            const int c = e / TNB, r = e % TNB;  // column c, row r of the diagonal block
            Ld[r][c] = L[(int64_t)(J + c) * B + J + r];
        }
        __syncthreads();
        if (tid < TSH) {
            // row tid: x_c = (t_c - Σ_{d<c} x_d L[c][d]) / L[c][c]
#pragma unroll
            for (int c = 0; c < TNB; ++c) {
                double v = T[tid][c];
#pragma unroll
                for (int d = 0; d < c; ++d) v -= T[tid][d] * Ld[c][d];
                T[tid][c] = v / Ld[c][c];
            }
        }
        __syncthreads();
        for (int e = tid; e < TSH * TNB; e += 256) {
            const int c = e / TSH, r = e % TSH;
            X[(int64_t)(J + c) * B + r0 + r] = T[r][c];
        }
        __syncthreads();
    }
}

void launch_trsm(double *tiles, int b, int64_t nt, int64_t k, const int64_t *info, hipStream_t s)
{
    const int64_t m = nt - k - 1;
    if (m <= 0) return;
    dim3 grid((unsigned)m, (unsigned)(b / TSH));
    switch (b) {
    case 128: trsm_kernel<128><<<grid, 256, 0, s>>>(tiles, k, info); break;
    case 256: trsm_kernel<256><<<grid, 256, 0, s>>>(tiles, k, info); break;
    case 384: trsm_kernel<384><<<grid, 256, 0, s>>>(tiles, k, info); break;
    default: trsm_kernel<512><<<grid, 256, 0, s>>>(tiles, k, info); break;
    }
}

}  // namespace gl
