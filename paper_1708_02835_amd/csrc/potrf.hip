// Diagonal-tile Cholesky factorisation (the POTRF task of the tile algorithm,
// Sec. 5.2 and Alg. 2 step 3).
//
// One workgroup of 256 threads factors the b×b tile A_kk = L_kk L_kkᵀ in place
// (lower triangle), right-looking over 64-column panels s:
//   1. the 64×64 diagonal block D is copied to LDS, factored and inverted in
//      16×16 sub-blocks (factor_invert_64: small scalar factorisations and
//      inverses of the diagonal sub-blocks, everything else on the matrix
//      cores).  D⁻¹ is also written to `dinv` for the panel TRSM and the
//      forward solve of this step;
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
// At b = 128 the whole tile stays in LDS between the steps (potrf_tile128).
// The kernel runs beside the bulk trailing updates, so it starts only when a
// CU has room for its registers and LDS: its footprint is kept at what the
// general path needs (a fully unrolled block read raised the registers and
// made some calls wait out a whole trailing launch).
#include "batch.hpp"
#include "common.hpp"
#include "mfma.hpp"

namespace gl {

constexpr int PB = 64;  // diagonal block edge

// d = sqrt(p) and inv = 1/sqrt(p) for a pivot p > 0.  The generic binary64
// square root and division are long dependent sequences on the critical
// chain of the column loop below; here the hardware reciprocal square root
// (about 2^-23 relative error) is refined by two coupled Newton steps of
// Goldschmidt's iteration, g -> sqrt(p) and h -> 1/(2 sqrt(p)), each of which
// squares the relative error, and the root gets one residual correction
// d = g + (p - g²) h (Markstein's final step).  Both results are within a
// few ulps of the correctly rounded values, well inside the spread of other
// binary64 orderings of the factorisation.
__device__ __forceinline__ void pivot_root(double p, double &d, double &inv)
{
    const double y = __builtin_amdgcn_rsq(p);
    double g = p * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    d = fma(fma(-g, g, p), h, g);
    inv = h + h;
}

// Factor the 64×64 block D held in Ds (Ds[c][r] = D[r][c], lower triangle
// valid) as D = L Lᵀ in place and write X = L⁻¹ to Xi (Xi[c][r] = X[r][c];
// its upper blocks must be zero on entry), in 16×16 sub-blocks, P = 0..3:
//   (a) one wave factors the 16×16 diagonal block D_PP (lane r owns row r,
//       each column broadcast through LDS) and inverts it (lane j builds
//       column j of X_PP by forward substitution);
//   (b) the blocks below, L_IP = D_IP X_PPᵀ, on the matrix cores, one wave
//       per block;
//   (c) the lower blocks to the right, D_IJ -= L_IP L_JPᵀ (P < J <= I), on
//       the matrix cores.
// Then the off-diagonal blocks of X by block diagonals d = I - J = 1, 2, 3:
// X_IJ = -X_II Σ_{M=J}^{I-1} L_IM X_MJ.  The 16x16x4 products leave T = Σ
// in the lane layout of their B operand, so the second product reads it from
// registers.  A non-positive (or NaN) pivot stores the 1-based global column
// (col0 + local column + 1) in *info; the function returns false on every
// thread in that case and true otherwise.  Called by all 256 threads.
__device__ __forceinline__ bool factor_invert_64(double (*Ds)[PB + 1], double (*Xi)[PB + 1], double *rdiag,
                                                 double *colb, int *fail, int64_t col0, int64_t *info)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int r16 = lane & 15;  // row (column) within a 16×16 block
    const int q = lane >> 4;
    for (int P = 0; P < 4; ++P) {
        const int p0 = 16 * P;
        if (wave == 0) {
            // (a) lanes 16..63 repeat the work of lanes 0..15 and store nothing
            double a[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) a[m] = Ds[p0 + m][p0 + r16];
            int fcol = -1;
            double rv = 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const double piv = readlane_f64(a[c], c);
                if (!(piv > 0.0) && fcol < 0) fcol = c;
                double d, inv;
                pivot_root(piv, d, inv);
                if (r16 == c) rv = inv;
                a[c] = (r16 == c) ? d : a[c] * inv;
                // column c through LDS (the wave's LDS accesses complete in
                // order); entries above the diagonal receive values that are
                // never stored
                if (lane < 16) colb[lane] = a[c];
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int j = c + 1; j < 16; ++j) a[j] -= a[c] * colb[j];
                __builtin_amdgcn_wave_barrier();
            }
            if (fcol >= 0) {
                if (lane == 0) {
                    *fail = 1;
                    *info = col0 + p0 + fcol + 1;
                }
            } else {
                if (lane < 16) {
#pragma unroll
                    for (int m = 0; m < 16; ++m)
                        if (m <= lane) Ds[p0 + m][p0 + lane] = a[m];
                    rdiag[p0 + lane] = rv;
                }
                __builtin_amdgcn_wave_barrier();
                double x[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) x[i] = (i == r16) ? 1.0 : 0.0;
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    x[m] *= rdiag[p0 + m];
#pragma unroll
                    for (int i = m + 1; i < 16; ++i) x[i] -= Ds[p0 + m][p0 + i] * x[m];
                }
                if (lane < 16) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) Xi[p0 + lane][p0 + i] = x[i];
                }
            }
        }
        __syncthreads();
        if (*fail) return false;  // uniform: shared flag read after the barrier
        if (wave < 3 - P) {
            // (b) block I = P + 1 + wave: L_IP[i][j] = Σ_m D_IP[i][m] X_PP[j][m]
            const int i0 = 16 * (P + 1 + wave);
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                const int m = 4 * kc + q;
                acc = mfma_f64(Ds[p0 + m][i0 + r16], Xi[p0 + m][p0 + r16], acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) Ds[p0 + r16][i0 + q + 4 * r] = acc[r];
        }
        __syncthreads();
        const int nb = 3 - P;
        for (int blk = wave; blk < nb * (nb + 1) / 2; blk += 4) {
            // (c) block (I, J), P < J <= I
            int bi = 0;
            while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
            const int bj = blk - bi * (bi + 1) / 2;
            const int i0 = 16 * (P + 1 + bi), j0 = 16 * (P + 1 + bj);
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                const int m = 4 * kc + q;
                acc = mfma_f64(Ds[p0 + m][i0 + r16], Ds[p0 + m][j0 + r16], acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) Ds[j0 + r16][i0 + q + 4 * r] -= acc[r];
        }
        __syncthreads();
    }
    for (int dd = 1; dd < 4; ++dd) {
        if (wave < 4 - dd) {
            const int J = wave, I = wave + dd;
            d4 t = {0.0, 0.0, 0.0, 0.0};
            for (int M = J; M < I; ++M) {
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    const int m = 4 * kc + q;
                    t = mfma_f64(Ds[16 * M + m][16 * I + r16], Xi[16 * J + r16][16 * M + m], t);
                }
            }
            d4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) x = mfma_f64(Xi[16 * I + 4 * kc + q][16 * I + r16], t[kc], x);
#pragma unroll
            for (int r = 0; r < 4; ++r) Xi[16 * J + r16][16 * I + q + 4 * r] = -x[r];
        }
        __syncthreads();
    }
    return true;
}

// b = 128: the whole lower tile fits in LDS (three 64×64 blocks: D0, the
// rows below it, D1), so it is read once, both panels are factored there and
// only the results go back; the steps and their arithmetic are those of
// potrf_general below (a panel solve and one trailing update between the two
// diagonal blocks), without the global-memory round trips between them.
__device__ __forceinline__ void potrf_tile128(double *__restrict__ tiles, int64_t k, int64_t n,
                                              int64_t *__restrict__ info, double *__restrict__ logsum,
                                              double *__restrict__ dinv)
{
    constexpr int B = 128;
    double *A = tiles + tile_offset(k, k, B);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    __shared__ double D0[PB][PB + 1];  // D0[c][r] = A[r][c]: first diagonal block, then L0
    __shared__ double Pn[PB][PB + 1];  // Pn[c][r] = A[64 + r][c]: rows below, then the panel P
    __shared__ double D1[PB][PB + 1];  // D1[c][r] = A[64 + r][64 + c]: second diagonal block
    __shared__ double Xi[PB][PB + 1];
    __shared__ double rdiag[PB];
    __shared__ double colb[16];
    __shared__ double red[4];
    __shared__ int fail;

    for (int e = tid; e < PB * PB; e += 256) {
        const int c = e >> 6, r = e & 63;
        D0[c][r] = A[(int64_t)c * B + r];
        Pn[c][r] = A[(int64_t)c * B + PB + r];
        D1[c][r] = A[(int64_t)(PB + c) * B + PB + r];
        Xi[c][r] = 0.0;
    }
    if (tid == 0) fail = 0;
    __syncthreads();
    if (!factor_invert_64(D0, Xi, rdiag, colb, &fail, k * B, info)) return;
    for (int e = tid; e < PB * PB; e += 256) {
        const int c = e >> 6, r = e & 63;
        if (r >= c) A[(int64_t)c * B + r] = D0[c][r];
        dinv[c * PB + r] = Xi[c][r];
    }
    {
        // panel P = A[64:128, 0:64] · D0⁻ᵀ, wave w owning rows 16w..16w+15; each
        // wave reads its own rows of Pn before writing them
        const int r0 = wave * 16;
        double y[PB / 4];
#pragma unroll
        for (int kk = 0; kk < PB / 4; ++kk) y[kk] = Pn[4 * kk + (lane >> 4)][r0 + (lane & 15)];
        d4 acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            acc[cb] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < PB / 4; ++kk)
                acc[cb] = mfma_f64(Xi[4 * kk + (lane >> 4)][cb * 16 + (lane & 15)], y[kk], acc[cb]);
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = cb * 16 + mfma_row(lane, q), r = r0 + mfma_col(lane);
                A[(int64_t)c * B + PB + r] = acc[cb][q];
                Pn[c][r] = acc[cb][q];
            }
    }
    __syncthreads();
    // D1 -= P Pᵀ, lower triangle, in 32×32 blocks (0,0), (1,0), (1,1), K = 64 in two halves
    if (wave < 3) {
        const int bi = wave == 0 ? 0 : 1, bj = wave == 2 ? 1 : 0;
        const int ra = bi * 32 + (lane & 15), rc = bj * 32 + (lane & 15);
        d4 c00 = {0.0, 0.0, 0.0, 0.0}, c01 = c00, c10 = c00, c11 = c00;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            double a0[8], a1[8], b0[8], b1[8];
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int col = 32 * h + 4 * kk + (lane >> 4);
                a0[kk] = Pn[col][ra];
                a1[kk] = Pn[col][ra + 16];
                b0[kk] = Pn[col][rc];
                b1[kk] = Pn[col][rc + 16];
            }
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                c00 = mfma_f64(b0[kk], a0[kk], c00);
                c01 = mfma_f64(b1[kk], a0[kk], c01);
                c10 = mfma_f64(b0[kk], a1[kk], c10);
                c11 = mfma_f64(b1[kk], a1[kk], c11);
            }
        }
        const int rr = bi * 32 + mfma_col(lane), cc = bj * 32;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int col = cc + mfma_row(lane, q);
            D1[col][rr] -= c00[q];
            D1[col + 16][rr] -= c01[q];
            D1[col][rr + 16] -= c10[q];
            D1[col + 16][rr + 16] -= c11[q];
        }
    }
    for (int e = tid; e < PB * PB; e += 256) Xi[e >> 6][e & 63] = 0.0;
    __syncthreads();
    if (!factor_invert_64(D1, Xi, rdiag, colb, &fail, k * B + PB, info)) return;
    for (int e = tid; e < PB * PB; e += 256) {
        const int c = e >> 6, r = e & 63;
        if (r >= c) A[(int64_t)(PB + c) * B + PB + r] = D1[c][r];
        dinv[PB * PB + c * PB + r] = Xi[c][r];
    }
    // 2 Σ log L_rr over the rows that are not padding
    double acc = 0.0;
    if (tid < B && k * B + tid < n) acc = log(tid < PB ? D0[tid][tid] : D1[tid - PB][tid - PB]);
    double w = wave_sum(acc);
    if (lane == 0) red[wave] = w;
    __syncthreads();
    if (tid == 0) logsum[k] = 2.0 * ((red[0] + red[1]) + (red[2] + red[3]));
}

template <int B>
__device__ __forceinline__ void potrf_general(double *__restrict__ tiles, int64_t k, int64_t n,
                                              int64_t *__restrict__ info, double *__restrict__ logsum,
                                              double *__restrict__ dinv)
{
    double *A = tiles + tile_offset(k, k, B);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    __shared__ double Ds[PB][PB + 1];  // Ds[c][r] = D[r][c]
    __shared__ double Xi[PB][PB + 1];  // Xi[c][r] = (D⁻¹)[r][c]
    __shared__ double rdiag[PB];
    __shared__ double colb[16];  // the current column of a 16×16 factor, for broadcast reads
    __shared__ double red[4];
    __shared__ int fail;

    for (int s = 0; s < B; s += PB) {
        for (int e = tid; e < PB * PB; e += 256) {
            const int c = e >> 6, r = e & 63;
            Ds[c][r] = A[(int64_t)(s + c) * B + s + r];
            Xi[c][r] = 0.0;  // D⁻¹ is lower triangular: the upper blocks stay zero
        }
        if (tid == 0) fail = 0;
        __syncthreads();
        if (!factor_invert_64(Ds, Xi, rdiag, colb, &fail, k * B + s, info)) return;
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
__device__ __forceinline__ void potrf_body(double *__restrict__ tiles, int64_t k, int64_t n,
                                           int64_t *__restrict__ info, double *__restrict__ logsum,
                                           double *__restrict__ dinv)
{
    if (*info != 0) return;
    __builtin_amdgcn_s_setprio(3);  // critical path of the step schedule
    if constexpr (B == 128) potrf_tile128(tiles, k, n, info, logsum, dinv);
    else potrf_general<B>(tiles, k, n, info, logsum, dinv);
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
