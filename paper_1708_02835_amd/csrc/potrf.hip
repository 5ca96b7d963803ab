// Diagonal-tile Cholesky factorisation (the POTRF task of the tile algorithm,
// Sec. 5.2 and Alg. 2 step 3).
//
// One workgroup of 256 threads factors the b×b tile A_kk = L_kk L_kkᵀ in place
// (lower triangle), right-looking over 64-column panels s:
//   1. the 64×64 diagonal block D is copied to LDS, factored by one wave
//      (lane r owns row r; each column of the factor is broadcast through
//      LDS), and inverted by the same wave (lane j builds column j of D⁻¹ by
//      column-oriented forward substitution).  D⁻¹ is also written to `dinv` for the panel TRSM and
//      the forward solve of this step;
//   2. the rows below the block are solved on the matrix cores as
//      P = A[s+64:, s:s+64] · D⁻ᵀ, each wave owning whole 16-row groups;
//   3. the trailing lower triangle A[s+64:, s+64:] -= P Pᵀ is updated on the
//      matrix cores in 32×32 blocks shared by the four waves.
// Applying inverted 64×64 diagonal blocks instead of substituting element by
// element is the usual GPU form of the blocked triangular solve; its rounding
// stays within the spread of other binary64 orderings (see the parity tests).
// A non-positive (or NaN) pivot stores the 1-based global column in *info and
// stops; every later kernel of the factorisation then returns immediately.
// The tile's contribution 2 Σ log L_rr over rows r < n goes to logsum[k].
#include "batch.hpp"
#include "common.hpp"
#include "mfma.hpp"

namespace gl {

constexpr int PB = 64;  // diagonal block edge

template <int B>
__device__ __forceinline__ void potrf_body(double *__restrict__ tiles, int64_t k, int64_t n,
                                           int64_t *__restrict__ info, double *__restrict__ logsum,
                                           double *__restrict__ dinv)
{
    if (*info != 0) return;
    __builtin_amdgcn_s_setprio(3);  // critical path of the step schedule
    double *A = tiles + tile_offset(k, k, B);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    __shared__ double Ds[PB][PB + 1];  // Ds[c][r] = D[r][c]
    __shared__ double Xi[PB][PB + 1];  // Xi[c][r] = (D⁻¹)[r][c]
    __shared__ double rdiag[PB];
    __shared__ double colb[PB];  // the current column of the 64×64 factor, for broadcast reads
    __shared__ double red[4];
    __shared__ int fail;

    for (int s = 0; s < B; s += PB) {
        for (int e = tid; e < PB * PB; e += 256) {
            const int c = e >> 6, r = e & 63;
            Ds[c][r] = A[(int64_t)(s + c) * B + s + r];
        }
        if (tid == 0) fail = 0;
        __syncthreads();
        if (wave == 0) {
            // unblocked right-looking Cholesky of D with row `lane` in registers;
            // the pivot and the column multipliers are broadcast by readlane
            double a[PB];
#pragma unroll
            for (int m = 0; m < PB; ++m) a[m] = Ds[m][lane];
            int fcol = -1;
            double rv = 0.0;
#pragma unroll
            for (int c = 0; c < PB; ++c) {
                const double piv = readlane_f64(a[c], c);
                if (!(piv > 0.0) && fcol < 0) fcol = c;
                const double d = sqrt(piv);
                const double inv = 1.0 / d;
                if (lane == c) rv = inv;
                a[c] = (lane == c) ? d : a[c] * inv;
                // column c goes through LDS (one store, then broadcast reads: the
                // wave's LDS accesses complete in order) for the rank-1 update;
                // entries above the diagonal (lane < j) receive harmless values
                // that are never stored
                colb[lane] = a[c];
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int j = c + 1; j < PB; ++j) a[j] -= a[c] * colb[j];
                __builtin_amdgcn_wave_barrier();
            }
            if (fcol >= 0) {
                if (lane == 0) {
                    fail = 1;
                    *info = k * B + s + fcol + 1;
                }
            } else {
#pragma unroll
                for (int m = 0; m < PB; ++m) Ds[m][lane] = a[m];
                rdiag[lane] = rv;
            }
        }
        __syncthreads();
        if (fail) return;  // uniform: shared flag read after the barrier
        if (wave == 0) {
            // column `lane` of D⁻¹: X[i][j] = (δ_ij - Σ_{m<i} D[i][m] X[m][j]) / D[i][i],
            // column-oriented: once X[m][j] is final it is subtracted from every
            // later row, so the updates of one step are independent (the same
            // operations in the same order per entry as row by row)
            double x[PB];
#pragma unroll
            for (int i = 0; i < PB; ++i) x[i] = (i == lane) ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < PB; ++m) {
                x[m] *= rdiag[m];
#pragma unroll
                for (int i = m + 1; i < PB; ++i) x[i] -= Ds[m][i] * x[m];
            }
#pragma unroll
            for (int i = 0; i < PB; ++i) Xi[lane][i] = x[i];
        }
        __syncthreads();
        // L block back to the tile, D⁻¹ to the step's inverse buffer
        double *dv = dinv + (int64_t)(s / PB) * PB * PB;
        for (int e = tid; e < PB * PB; e += 256) {
            const int c = e >> 6, r = e & 63;
            if (r >= c) A[(int64_t)(s + c) * B + s + r] = Ds[c][r];
            dv[c * PB + r] = Xi[c][r];
        }
        // panel rows below: P = A[s+64:, s:s+64] · D⁻ᵀ
        const int R = B - s - PB;
        for (int rb = wave; rb < R / 16; rb += 4) {
            const int r0 = s + PB + rb * 16;
            double y[PB / 4];
#pragma unroll
            for (int kk = 0; kk < PB / 4; ++kk)
                y[kk] = A[(int64_t)(s + 4 * kk + (lane >> 4)) * B + r0 + (lane & 15)];
            d4 acc[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                acc[cb] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < PB / 4; ++kk)
                    acc[cb] = mfma_f64(Xi[4 * kk + (lane >> 4)][cb * 16 + (lane & 15)], y[kk], acc[cb]);
            }
            // result row q of lane l: column cb*16 + l/16 + 4q; lane % 16: row
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    A[(int64_t)(s + cb * 16 + mfma_row(lane, q)) * B + r0 + mfma_col(lane)] = acc[cb][q];
        }
        __syncthreads();
        // trailing lower triangle in 32×32 blocks, K = 64 in two halves
        if (R > 0) {
            const int nb = R / 32;
            const int nblk = nb * (nb + 1) / 2;
            const int t0 = s + PB;
            for (int blk = wave; blk < nblk; blk += 4) {
                int bi = (int)((sqrt(8.0 * blk + 1.0) - 1.0) * 0.5);
                while (bi * (bi + 1) / 2 > blk) --bi;
                while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
                const int bj = blk - bi * (bi + 1) / 2;
                const int ra = t0 + bi * 32 + (lane & 15);  // C rows
                const int rc = t0 + bj * 32 + (lane & 15);  // C columns
                d4 c00 = {0.0, 0.0, 0.0, 0.0}, c01 = c00, c10 = c00, c11 = c00;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    double a0[8], a1[8], b0[8], b1[8];
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk) {
                        const int64_t col = s + 32 * h + 4 * kk + (lane >> 4);
                        a0[kk] = A[col * B + ra];
                        a1[kk] = A[col * B + ra + 16];
                        b0[kk] = A[col * B + rc];
                        b1[kk] = A[col * B + rc + 16];
                    }
                    // operands swapped: result row = C column, lane % 16 = C row
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk) {
                        c00 = mfma_f64(b0[kk], a0[kk], c00);
                        c01 = mfma_f64(b1[kk], a0[kk], c01);
                        c10 = mfma_f64(b0[kk], a1[kk], c10);
                        c11 = mfma_f64(b1[kk], a1[kk], c11);
                    }
                }
                const int rr = t0 + bi * 32 + mfma_col(lane);
                const int cc = t0 + bj * 32;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t col = cc + mfma_row(lane, q);
                    A[col * B + rr] -= c00[q];
                    A[(col + 16) * B + rr] -= c01[q];
                    A[col * B + rr + 16] -= c10[q];
                    A[(col + 16) * B + rr + 16] -= c11[q];
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

template <int B>
__global__ __launch_bounds__(256) void potrf_kernel(double *__restrict__ tiles, int64_t k, int64_t n,
                                                    int64_t *__restrict__ info,
                                                    double *__restrict__ logsum,
                                                    double *__restrict__ dinv)
{
    potrf_body<B>(tiles, k, n, info, logsum, dinv);
}

void launch_potrf(double *tiles, int b, int64_t k, int64_t n, int64_t *info, double *logsum,
                  double *dinv, hipStream_t s)
{
    switch (b) {
    case 128: potrf_kernel<128><<<1, 256, 0, s>>>(tiles, k, n, info, logsum, dinv); break;
    case 256: potrf_kernel<256><<<1, 256, 0, s>>>(tiles, k, n, info, logsum, dinv); break;
    case 384: potrf_kernel<384><<<1, 256, 0, s>>>(tiles, k, n, info, logsum, dinv); break;
    default: potrf_kernel<512><<<1, 256, 0, s>>>(tiles, k, n, info, logsum, dinv); break;
    }
}

template <int B>
__global__ __launch_bounds__(256) void potrf_batched_kernel(const BatchReq *__restrict__ d)
{
    const BatchReq &r = d[blockIdx.x];
    potrf_body<B>(r.tiles, r.k, r.n, r.info, r.logsum, r.dinv);
}

void launch_potrf_batched(int b, const BatchReq *d, int count, hipStream_t s)
{
    switch (b) {
    case 128: potrf_batched_kernel<128><<<count, 256, 0, s>>>(d); break;
    case 256: potrf_batched_kernel<256><<<count, 256, 0, s>>>(d); break;
    case 384: potrf_batched_kernel<384><<<count, 256, 0, s>>>(d); break;
    default: potrf_batched_kernel<512><<<count, 256, 0, s>>>(d); break;
    }
}

}  // namespace gl
