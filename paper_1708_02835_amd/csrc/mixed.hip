// Mixed-precision tiled Cholesky: per-tile precision of the trailing update.
//
// Every tile is stored in binary64 and the diagonal tiles, POTRF, TRSM, the
// solve and the log-determinant stay binary64.  What changes is the precision
// of the trailing products A_ij -= L_ik L_jkᵀ of off-band tiles, chosen per
// tile (i, j) from the normalised tile norm
//     ν_ij = ||Σ_ij||_F / sqrt(||Σ_ii||_F ||Σ_jj||_F)
// measured when Σ is generated:
//   class 0  FP64    diagonal tiles, tiles with i - j < band, and tiles
//                    with ν_ij > tol_64 (both modes);
//   class 1  FP32    FP32 matrix-core products (GL_MIXED_FP32);
//   class 2  BF16x6  operands split into three bfloat16 parts a = h + m + l,
//                    products hh + hm + mh + hl + lh + mm: about FP32 accuracy
//                    (GL_MIXED_BF16, ν_ij > tol_hi);
//   class 3  BF16x3  two parts, products hh + hm + mh (tol_lo < ν_ij <= tol_hi);
//   class 4  BF16    one part (ν_ij <= tol_lo);
//   class 5  FP16x3  (GL_MIXED_FP16) operands scaled by s = 2^e so that
//                    |L_ik| <= sqrt(max(θ1, 1)) maps below 2^14, split in two
//                    binary16 parts a = h + l, products hh + hl + lh (about 22
//                    bits; ν_ij > tol_lo), the FP32 result times s⁻²;
//   class 6  FP16    one scaled binary16 part (ν_ij <= tol_lo).
// Binary16 carries 11 bits against bfloat16's 8, so with the scale keeping
// every panel value inside its range, two parts and three products reach the
// accuracy for which bfloat16 needs three parts and six products.  Values far
// below the scale lose relative precision (subnormal low parts), but only at
// an absolute level of 2^-39 sqrt(max(θ1, 1)).
// Thresholds left negative in the options follow from an accuracy target
// and the first diagonal tile's pivots (thresholds_kernel below).
// Low-precision products accumulate in FP32 over the whole K = b of one tile
// update and are subtracted from an FP32 running sum of the tile's updates
// (half the bytes of a binary64 read-modify-write per update); the sum is
// added to the binary64 tile once, when the tile's column becomes the panel
// (before its TRSM).
// The split-bfloat16 products follow Henry, Tang and Heinecke, "Leveraging the
// bfloat16 artificial intelligence datatype for higher-precision
// computations" (ARITH 2019).
//
// After the TRSM of step k, the panel column L_ik (i > k) is copied into the
// formats the classes need: FP32 column-major, or bfloat16 parts stored
// row-major (k contiguous, the operand layout of the BF16 matrix-core
// product).  Copies are double-buffered by the parity of k, so the bulk
// update of step k can still read them while step k+1 writes its own.
#include <algorithm>
#include <cmath>
#include <vector>

#include "engine.hpp"
#include "mfma.hpp"

namespace gl {

enum { C64 = 0, C32 = 1, CB6 = 2, CB3 = 3, CB1 = 4, CH2 = 5, CH1 = 6, NCLASS = GL_NCLASS };
static_assert(NCLASS == 7, "class count");

// ------------------------------------------------------------ precision map --

// Smallest pivot ratio ρ = min_r L_rr² / θ1 of the first diagonal tile,
// factored in binary64 before any off-band update (Σ_rr = θ1).  It measures
// how much of a variance the neighbouring locations explain, i.e. how much
// the Schur complements cancel; a non-positive or NaN ρ (failed POTRF) makes
// every adaptive threshold zero, so every tile stays binary64.  Then the
// effective thresholds: a negative option is replaced by ε ρ / u for the
// class it bounds (u = 2⁻²⁴ for FP32 and the three-part split, 2⁻¹⁶ for two
// bfloat16 parts, 2⁻⁸ for one; 2⁻²² for two binary16 parts, 2⁻¹¹ for one),
// i.e. a class is used for tile (i, j) only while ν_ij u <= ε ρ.
// thr = {ρ, tol_64, tol_hi, tol_lo}; the FP16 mode has no tol_hi class and
// reports tol_64 there.
__global__ __launch_bounds__(256) void thresholds_kernel(const double *__restrict__ tile0, int b, int64_t n,
                                                         double theta1, int mode, double eps, double tol_64,
                                                         double tol_hi, double tol_lo, double *__restrict__ thr)
{
    const int m = (int)(n < b ? n : b);
    double lo = INFINITY;
    for (int r = threadIdx.x; r < m; r += 256) {
        const double d = tile0[(int64_t)r * b + r];
        lo = fmin(lo, d * d / theta1);
    }
    for (int off = 32; off >= 1; off >>= 1) lo = fmin(lo, __shfl_xor(lo, off, 64));
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lo;
    __syncthreads();
    if (threadIdx.x == 0) {
        double rho = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
        if (!(rho > 0.0) || !(rho <= 1.0)) rho = 0.0;
        const double er = eps * rho;
        thr[0] = rho;
        if (mode == GL_MIXED_FP16) {
            thr[1] = tol_64 >= 0.0 ? tol_64 : er * 4194304.0;  // / 2^-22
            thr[2] = thr[1];
            thr[3] = tol_lo >= 0.0 ? tol_lo : er * 2048.0;     // / 2^-11
        } else {
            thr[1] = tol_64 >= 0.0 ? tol_64 : er * 16777216.0;  // / 2^-24
            thr[2] = tol_hi >= 0.0 ? tol_hi : er * 65536.0;     // / 2^-16
            thr[3] = tol_lo >= 0.0 ? tol_lo : er * 256.0;       // / 2^-8
        }
    }
}

__global__ void classify_kernel(const double *__restrict__ norm2, int64_t nt, int band, int mode,
                                const double *__restrict__ thr, uint8_t *__restrict__ map)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= tile_count(nt)) return;
    int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > t) --i;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    const int64_t j = t - i * (i + 1) / 2;
    const double tol_64 = thr[1], tol_hi = thr[2], tol_lo = thr[3];
    uint8_t c;
    if (i - j < band) {
        c = C64;
    } else {
        const double nij = sqrt(norm2[t]);
        const double nii = sqrt(norm2[tile_index(i, i)]);
        const double njj = sqrt(norm2[tile_index(j, j)]);
        const double v = nij / sqrt(nii * njj);
        if (!(v <= tol_64)) c = C64;
        else if (mode == GL_MIXED_FP32) c = C32;
        else if (mode == GL_MIXED_FP16) c = (v > tol_lo) ? CH2 : CH1;
        else c = (v > tol_hi) ? CB6 : (v > tol_lo) ? CB3 : CB1;
    }
    map[t] = c;
}

// --------------------------------------------------------------- bfloat16 --

// Round to nearest even (finite inputs).
__device__ inline uint16_t bf16_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_value(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ inline uint16_t f16_bits(_Float16 h)
{
    uint16_t u;
    __builtin_memcpy(&u, &h, sizeof(u));
    return u;
}

// Panel copies of step k.  Workgroup (tile i, 64×64 block): reads the binary64
// block of L_ik and writes the FP32 copy (column-major), or np parts (row-major,
// via an LDS transpose): bfloat16 parts when f16s = 0, else the two binary16
// parts of s L_ik, s = f16s (a power of two, so the scaling is exact; the
// residual of the first part is exact in FP32).
template <int B>
__global__ __launch_bounds__(256) void panel_convert_kernel(const double *__restrict__ tiles, int64_t k,
                                                            float *__restrict__ p32,
                                                            uint16_t *__restrict__ planes,
                                                            int64_t plane_stride, int np, float f16s,
                                                            const int64_t *__restrict__ info)
{
    if (*info != 0) return;
    const int64_t i = k + 1 + blockIdx.x;
    const int bi = blockIdx.y / (B / 64), bj = blockIdx.y % (B / 64);  // row block, column block
    const double *L = tiles + tile_offset(i, k, B);
    const int tid = threadIdx.x;
    if (p32) {
        float *P = p32 + i * (int64_t)B * B;
        for (int e = tid; e < 64 * 64; e += 256) {
            const int c = e >> 6, r = e & 63;
            const int64_t off = (int64_t)(bj * 64 + c) * B + bi * 64 + r;
            P[off] = (float)L[off];
        }
    }
    if (planes) {
        __shared__ float T[64][65];  // T[r][c]
        for (int e = tid; e < 64 * 64; e += 256) {
            const int c = e >> 6, r = e & 63;
            T[r][c] = (float)L[(int64_t)(bj * 64 + c) * B + bi * 64 + r];
        }
        __syncthreads();
        for (int e = tid; e < 64 * 64; e += 256) {
            const int r = e >> 6, c = e & 63;  // write row-major: consecutive threads, consecutive c
            const int64_t off = i * (int64_t)B * B + (int64_t)(bi * 64 + r) * B + bj * 64 + c;
            float v = T[r][c];
            if (f16s > 0.0f) {
                v *= f16s;
                const _Float16 h = (_Float16)v;
                planes[off] = f16_bits(h);
                planes[plane_stride + off] = f16_bits((_Float16)(v - (float)h));
                continue;
            }
            for (int p = 0; p < np; ++p) {
                const uint16_t h = bf16_bits(v);
                planes[p * plane_stride + off] = h;
                v = v - bf16_value(h);
            }
        }
    }
}

// ------------------------------------------------- FP32 trailing update --

constexpr int FB = 128;  // output block
constexpr int FK = 32;   // k chunk (eight 16x16x4 steps)

__device__ inline void list_tile(const int2 *__restrict__ list, int64_t G, int64_t nblocks, int sub_per_tile,
                                 int64_t &t, int &sub, bool &valid)
{
    const int64_t g = blockIdx.x;
    const int64_t lid = (g & 7) * (G >> 3) + (g >> 3);  // XCD-contiguous logical order
    valid = lid < nblocks;
    t = lid / sub_per_tile;
    sub = (int)(lid % sub_per_tile);
}

template <int B>
__global__ __launch_bounds__(256, 2) void trailing_f32_kernel(float *__restrict__ delta,
                                                              const float *__restrict__ p32,
                                                              const int2 *__restrict__ list,
                                                              int64_t nblocks,
                                                              const int64_t *__restrict__ info,
                                                              int critical)
{
    if (*info != 0) return;
    if (critical) __builtin_amdgcn_s_setprio(3);
    constexpr int SB = B / FB;
    int64_t t;
    int sub;
    bool valid;
    list_tile(list, gridDim.x, nblocks, SB * SB, t, sub, valid);
    if (!valid) return;
    const int2 ij = list[t];
    const int rb = sub / SB, cb = sub % SB;
    const float *Ap = p32 + (int64_t)ij.x * B * B + rb * FB;
    const float *Bp = p32 + (int64_t)ij.y * B * B + cb * FB;
    float *C = delta + tile_offset(ij.x, ij.y, B) + (int64_t)(cb * FB) * B + rb * FB;

    __shared__ float As[2][FK][FB];
    __shared__ float Bs[2][FK][FB];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lc = tid >> 3;          // chunk column 0..31
    const int lr = (tid & 7) * 16;    // 16 consecutive rows
    typedef float f4v __attribute__((ext_vector_type(4)));

    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f4){0.f, 0.f, 0.f, 0.f};

    f4v ra[4], rbv[4];
    {
        const f4v *pa = reinterpret_cast<const f4v *>(Ap + (int64_t)lc * B + lr);
        const f4v *pb = reinterpret_cast<const f4v *>(Bp + (int64_t)lc * B + lr);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ra[q] = pa[q];
            rbv[q] = pb[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *reinterpret_cast<f4v *>(&As[0][lc][lr + 4 * q]) = ra[q];
            *reinterpret_cast<f4v *>(&Bs[0][lc][lr + 4 * q]) = rbv[q];
        }
    }
    __syncthreads();
    constexpr int NK = B / FK;
    for (int kc = 0; kc < NK; ++kc) {
        const int cur = kc & 1;
        if (kc + 1 < NK) {
            const int64_t col = (int64_t)(kc + 1) * FK + lc;
            const f4v *pa = reinterpret_cast<const f4v *>(Ap + col * B + lr);
            const f4v *pb = reinterpret_cast<const f4v *>(Bp + col * B + lr);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ra[q] = pa[q];
                rbv[q] = pb[q];
            }
        }
#pragma unroll
        for (int kk = 0; kk < FK; kk += 4) {
            float av[4], bv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                av[q] = As[cur][kk + (lane >> 4)][wm * 64 + q * 16 + (lane & 15)];
                bv[q] = Bs[cur][kk + (lane >> 4)][wn * 64 + q * 16 + (lane & 15)];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma_f32(bv[b], av[a], acc[a][b]);
        }
        if (kc + 1 < NK) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                *reinterpret_cast<f4v *>(&As[cur ^ 1][lc][lr + 4 * q]) = ra[q];
                *reinterpret_cast<f4v *>(&Bs[cur ^ 1][lc][lr + 4 * q]) = rbv[q];
            }
        }
        __syncthreads();
    }
    // result element r of lane l: C row = lane % 16, C column = 4 (l / 16) + r
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = wm * 64 + a * 16 + mfma_col(lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t col = wn * 64 + b * 16 + mfma32_row(lane, r);
                C[col * B + row] -= acc[a][b][r];
            }
        }
}

// ----------------------------------------------- BF16 trailing update ----

constexpr int HK = 32;        // k chunk = one 16x16x32 product
constexpr int HP = HK;        // LDS row: 32 bf16 = 64 bytes, no padding (the parts are swizzled)

// LDS layout of the staged operands.  Row r holds 32 consecutive k values as
// four 16-byte parts; logical part c of row r is stored at part
// c ^ ((r >> 1) & 3).  Measured on gfx950 (bank-conflict counters on the two
// access patterns alone): the stores (16 consecutive lanes per cycle, four
// lanes per row) fill the 64 four-byte banks once whatever the swizzle, and
// the 16x16x32 fragment reads (lane l: row l % 16, part l / 16; lanes
// 8c..8c+7 and 8c+16..8c+23 served together) hit 16 distinct bank quads.
// A plain 64-byte pitch has 4 conflict cycles per read, an 80-byte pitch 4
// per read and 8 per store.
__device__ __forceinline__ int swz_part(int row, int part) { return part ^ ((row >> 1) & 3); }

template <int B, int NP, bool F16>
__global__ __launch_bounds__(256, 2) void trailing_bf16_kernel(float *__restrict__ delta,
                                                               const uint16_t *__restrict__ planes,
                                                               const uint16_t *__restrict__ planes_prev,
                                                               int64_t plane_stride,
                                                               const int2 *__restrict__ list,
                                                               int64_t nblocks,
                                                               const int64_t *__restrict__ info,
                                                               int critical, float unscale)
{
    if (*info != 0) return;
    if (critical) __builtin_amdgcn_s_setprio(3);
    constexpr int SB = B / FB;
    int64_t t;
    int sub;
    bool valid;
    list_tile(list, gridDim.x, nblocks, SB * SB, t, sub, valid);
    if (!valid) return;
    const int2 ij = list[t];
    const int rb = sub / SB, cb = sub % SB;
    // row-major parts: element (r, kk) of tile slot s at s*B*B + r*B + kk.
    // With planes_prev (the parts of step k-1) the update covers both steps,
    // K = 2b: A_ij -= L_i,k-1 L_j,k-1ᵀ + L_ik L_jkᵀ, one running-sum update.
    const int64_t aoff = (int64_t)ij.x * B * B + (int64_t)(rb * FB) * B;
    const int64_t boff = (int64_t)ij.y * B * B + (int64_t)(cb * FB) * B;
    const uint16_t *first = planes_prev ? planes_prev : planes;
    float *C = delta + tile_offset(ij.x, ij.y, B) + (int64_t)(cb * FB) * B + rb * FB;

    __shared__ uint16_t As[NP][FB][HP];
    __shared__ uint16_t Bs[NP][FB][HP];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));

    // One part: little arithmetic per byte, so the running sum is read before
    // the k loop (overlapping the first operand loads) and the accumulators
    // start from it (times s² in the binary16 class: exact); the sum then
    // takes one FP32 rounding per product step, far below these classes' own
    // 2^-8 / 2^-11 grade.  Two or three parts: the products are summed from
    // zero and subtracted once, one rounding per update.
    const float upscale = F16 ? 1.0f / unscale : 1.0f;
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if constexpr (NP == 1) {
                const int row = wm * 64 + a * 16 + mfma_col(lane);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[a][b][r] = -C[(int64_t)(wn * 64 + b * 16 + mfma32_row(lane, r)) * B + row] * upscale;
            } else {
                acc[a][b] = (f4){0.f, 0.f, 0.f, 0.f};
            }
        }

    // loader: 128 rows × 32 bf16 per part and operand = 512 16-byte pieces, two per thread
    // two register sets (one or two parts): the chunk two steps ahead is in
    // flight while one is computed, so global latency is covered by two chunks
    // of products
    constexpr int NK = B / HK;  // chunks per step; even for every supported tile size
    const int NKT = planes_prev ? 2 * NK : NK;
    u4 ra0[NP][2], rb0[NP][2], ra1[NP][2], rb1[NP][2];
    auto load = [&](u4 (&ra)[NP][2], u4 (&rbv)[NP][2], int kc) {
        const bool second = kc >= NK;
        const uint16_t *P = second ? planes : first;
        const uint16_t *Ap = P + aoff, *Bp = P + boff;
        const int k0 = (second ? kc - NK : kc) * HK;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int piece = tid + 256 * h;
                const int row = piece >> 2, part = piece & 3;
                ra[p][h] = *reinterpret_cast<const u4 *>(Ap + p * plane_stride + (int64_t)row * B + k0 + part * 8);
                rbv[p][h] = *reinterpret_cast<const u4 *>(Bp + p * plane_stride + (int64_t)row * B + k0 + part * 8);
            }
    };
    auto store = [&](const u4 (&ra)[NP][2], const u4 (&rbv)[NP][2]) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int piece = tid + 256 * h;
                const int row = piece >> 2, part = swz_part(row, piece & 3);
                *reinterpret_cast<u4 *>(&As[p][row][part * 8]) = ra[p][h];
                *reinterpret_cast<u4 *>(&Bs[p][row][part * 8]) = rbv[p][h];
            }
    };
    // the same bits feed the bfloat16 or the binary16 matrix-core product
    auto mm = [](const bf16x8 &x, const bf16x8 &y, f4 c) {
        if constexpr (F16) return mfma_f16(__builtin_bit_cast(f16x8, x), __builtin_bit_cast(f16x8, y), c);
        else return mfma_bf16(x, y, c);
    };
    auto compute = [&]() {
        // fragments: 8 consecutive k of one row per lane
        bf16x8 af[NP][4], bfr[NP][4];
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ra_ = wm * 64 + q * 16 + (lane & 15), rb_ = wn * 64 + q * 16 + (lane & 15);
                af[p][q] = *reinterpret_cast<const bf16x8 *>(&As[p][ra_][8 * swz_part(ra_, lane >> 4)]);
                bfr[p][q] = *reinterpret_cast<const bf16x8 *>(&Bs[p][rb_][8 * swz_part(rb_, lane >> 4)]);
            }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                // operands swapped (B-part first): result row = C column, lane % 16 = C row
                acc[a][b] = mm(bfr[0][b], af[0][a], acc[a][b]);
                if (NP >= 2) {
                    acc[a][b] = mm(bfr[1][b], af[0][a], acc[a][b]);
                    acc[a][b] = mm(bfr[0][b], af[1][a], acc[a][b]);
                }
                if (NP >= 3) {
                    acc[a][b] = mm(bfr[2][b], af[0][a], acc[a][b]);
                    acc[a][b] = mm(bfr[0][b], af[2][a], acc[a][b]);
                    acc[a][b] = mm(bfr[1][b], af[1][a], acc[a][b]);
                }
            }
    };
    if constexpr (NP <= 2) {
        // two register sets: the chunk two steps ahead is in flight while one
        // is computed.  The prefetches are unconditional (the last chunk is
        // loaded again near the end and never stored): with a load count that
        // does not depend on the path, the wait before storing one register
        // set leaves the other set's loads in flight instead of draining them.
        // (Measured at n = 100,000: four sets, or the first loads issued set
        // by set, ran 1-5 % slower.)
        load(ra0, rb0, 0);
        load(ra1, rb1, 1);
        for (int kc = 0; kc < NKT; kc += 2) {
            store(ra0, rb0);
            __syncthreads();
            load(ra0, rb0, kc + 2 < NKT ? kc + 2 : NKT - 1);
            compute();
            __syncthreads();
            store(ra1, rb1);
            __syncthreads();
            load(ra1, rb1, kc + 3 < NKT ? kc + 3 : NKT - 1);
            compute();
            __syncthreads();
        }
    } else {
        // three parts: one register set (a second would spill)
        load(ra0, rb0, 0);
        for (int kc = 0; kc < NKT; ++kc) {
            store(ra0, rb0);
            __syncthreads();
            if (kc + 1 < NKT) load(ra0, rb0, kc + 1);
            compute();
            __syncthreads();
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = wm * 64 + a * 16 + mfma_col(lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t col = wn * 64 + b * 16 + mfma32_row(lane, r);
                const float v = F16 ? acc[a][b][r] * unscale : acc[a][b][r];  // exact: a power of two
                if constexpr (NP == 1) C[col * B + row] = -v;
                else C[col * B + row] -= v;
            }
        }
}

// ---------------------------------- wide two-part split-product update ----

// The same update for the two-part classes (BF16x3, FP16x3) with a 256×256
// output block per workgroup: 512 threads (one workgroup per CU, two waves
// per SIMD), eight waves of 128×64 in a 2×4 arrangement.  Every staged
// operand byte feeds twice the products of the 128×128 kernel above, whose
// operand streams bound it.  Staging: one register set holding the
// next-but-one chunk and two LDS buffers (128 KB), swizzled as above.
constexpr int WB = 256;

template <int B, bool F16>
__global__ __launch_bounds__(512, 1) void trailing_split2_wide_kernel(float *__restrict__ delta,
                                                                      const uint16_t *__restrict__ planes,
                                                                      const uint16_t *__restrict__ planes_prev,
                                                                      int64_t plane_stride,
                                                                      const int2 *__restrict__ list,
                                                                      int64_t nblocks,
                                                                      const int64_t *__restrict__ info,
                                                                      int critical, float unscale)
{
    if (*info != 0) return;
    if (critical) __builtin_amdgcn_s_setprio(3);
    constexpr int NP = 2;
    constexpr int SB = B / WB;
    int64_t t;
    int sub;
    bool valid;
    list_tile(list, gridDim.x, nblocks, SB * SB, t, sub, valid);
    if (!valid) return;
    const int2 ij = list[t];
    const int rb = sub / SB, cb = sub % SB;
    const int64_t aoff = (int64_t)ij.x * B * B + (int64_t)(rb * WB) * B;
    const int64_t boff = (int64_t)ij.y * B * B + (int64_t)(cb * WB) * B;
    const uint16_t *first = planes_prev ? planes_prev : planes;
    float *C = delta + tile_offset(ij.x, ij.y, B) + (int64_t)(cb * WB) * B + rb * WB;

    __shared__ uint16_t As[2][NP][WB][HP];
    __shared__ uint16_t Bs[2][NP][WB][HP];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;  // rows wm·128, columns wn·64
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));

    f4 acc[8][4];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f4){0.f, 0.f, 0.f, 0.f};

    // 256 rows × 4 pieces of 16 bytes per operand and part: two per thread
    constexpr int NK = B / HK;
    const int NKT = planes_prev ? 2 * NK : NK;
    u4 ra[NP][2], rbv[NP][2];
    auto load = [&](int kc) {
        const bool second = kc >= NK;
        const uint16_t *P = second ? planes : first;
        const uint16_t *Ap = P + aoff, *Bp = P + boff;
        const int k0 = (second ? kc - NK : kc) * HK;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int piece = tid + 512 * h;
                const int row = piece >> 2, part = piece & 3;
                ra[p][h] = *reinterpret_cast<const u4 *>(Ap + p * plane_stride + (int64_t)row * B + k0 + part * 8);
                rbv[p][h] = *reinterpret_cast<const u4 *>(Bp + p * plane_stride + (int64_t)row * B + k0 + part * 8);
            }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int piece = tid + 512 * h;
                const int row = piece >> 2, part = swz_part(row, piece & 3);
                *reinterpret_cast<u4 *>(&As[buf][p][row][part * 8]) = ra[p][h];
                *reinterpret_cast<u4 *>(&Bs[buf][p][row][part * 8]) = rbv[p][h];
            }
    };
    auto mm = [](const bf16x8 &x, const bf16x8 &y, f4 c) {
        if constexpr (F16) return mfma_f16(__builtin_bit_cast(f16x8, x), __builtin_bit_cast(f16x8, y), c);
        else return mfma_bf16(x, y, c);
    };
    auto frag = [&](const uint16_t (*S)[HP], int row0, int q) {
        const int r = row0 + q * 16 + (lane & 15);
        return *reinterpret_cast<const bf16x8 *>(&S[r][8 * swz_part(r, lane >> 4)]);
    };
    auto compute = [&](int buf) {
        // the wave's four B fragments of both parts stay in registers while
        // its eight A fragments of both parts stream past them: products
        // B_h A_h, B_l A_h, B_h A_l (operands swapped: result row = C column,
        // lane % 16 = C row); four independent products separate two updates
        // of one accumulator
        bf16x8 bh[4], bl[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bh[q] = frag(Bs[buf][0], wn * 64, q);
            bl[q] = frag(Bs[buf][1], wn * 64, q);
        }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const bf16x8 ah = frag(As[buf][0], wm * 128, a), al = frag(As[buf][1], wm * 128, a);
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = mm(bh[b], ah, acc[a][b]);
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = mm(bl[b], ah, acc[a][b]);
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = mm(bh[b], al, acc[a][b]);
        }
    };
    // chunk kc is computed from buffer kc & 1; the registers hold chunk kc + 1
    // while kc is computed and go to the other buffer after it
    load(0);
    store(0);
    load(NKT > 1 ? 1 : 0);
    __syncthreads();
    for (int kc = 0; kc < NKT; ++kc) {
        compute(kc & 1);
        __builtin_amdgcn_sched_barrier(0);
        if (kc + 1 < NKT) {
            store((kc + 1) & 1);
            load(kc + 2 < NKT ? kc + 2 : NKT - 1);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = wm * 128 + a * 16 + mfma_col(lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t col = wn * 64 + b * 16 + mfma32_row(lane, r);
                const float v = F16 ? acc[a][b][r] * unscale : acc[a][b][r];  // exact: a power of two
                C[col * B + row] -= v;
            }
        }
}

// ------------------------------------------------------------- launchers --

// Split-product classes (bfloat16 and binary16 parts) can take the updates of
// steps k-1 and k in one launch (pair = true: the parts of both panels are
// held, by parity); so can the binary64 class, whose panels stay in place in
// the tiles (one read and write of a C tile per two panels, as in the
// binary64 schedule).  FP32 tiles take one panel per step.
static bool paired_class(int cls) { return cls == C64 || cls >= CB6; }

template <int B>
static void launch_class(int cls, double *tiles, int64_t k, const MixedViews &mv, const int2 *list,
                         int64_t count, const int64_t *info, bool critical, bool pair, hipStream_t s)
{
    if (count <= 0) return;
    const int64_t sub = (int64_t)(B / FB) * (B / FB);
    const int64_t nblocks = count * sub;
    const unsigned grid = (unsigned)(ceil_div(nblocks, 8) * 8);
    const int crit = critical ? 1 : 0;
    const int par = (int)(k & 1);
    const uint16_t *prev = pair ? mv.planes[par ^ 1] : nullptr;
    switch (cls) {
    case C64:
        launch_trailing_list(tiles, B, k, list, count, info, critical, pair, s);
        break;
    case C32:
        trailing_f32_kernel<B><<<grid, 256, 0, s>>>(mv.delta, mv.p32[par], list, nblocks, info, crit);
        break;
    case CB6:
        trailing_bf16_kernel<B, 3, false><<<grid, 256, 0, s>>>(mv.delta, mv.planes[par], prev, mv.plane_stride, list,
                                                                 nblocks, info, crit, 1.0f);
        break;
    case CB3:
        if constexpr (B % WB == 0) {
            const int64_t wblocks = count * (B / WB) * (B / WB);
            trailing_split2_wide_kernel<B, false><<<(unsigned)(ceil_div(wblocks, 8) * 8), 512, 0, s>>>(
                mv.delta, mv.planes[par], prev, mv.plane_stride, list, wblocks, info, crit, 1.0f);
        } else {
            trailing_bf16_kernel<B, 2, false><<<grid, 256, 0, s>>>(mv.delta, mv.planes[par], prev, mv.plane_stride,
                                                                     list, nblocks, info, crit, 1.0f);
        }
        break;
    case CB1:
        trailing_bf16_kernel<B, 1, false><<<grid, 256, 0, s>>>(mv.delta, mv.planes[par], prev, mv.plane_stride, list,
                                                                 nblocks, info, crit, 1.0f);
        break;
    case CH2:
        if constexpr (B % WB == 0) {
            const int64_t wblocks = count * (B / WB) * (B / WB);
            trailing_split2_wide_kernel<B, true><<<(unsigned)(ceil_div(wblocks, 8) * 8), 512, 0, s>>>(
                mv.delta, mv.planes[par], prev, mv.plane_stride, list, wblocks, info, crit, mv.f16_unscale);
        } else {
            trailing_bf16_kernel<B, 2, true><<<grid, 256, 0, s>>>(mv.delta, mv.planes[par], prev, mv.plane_stride,
                                                                    list, nblocks, info, crit, mv.f16_unscale);
        }
        break;
    default:
        trailing_bf16_kernel<B, 1, true><<<grid, 256, 0, s>>>(mv.delta, mv.planes[par], prev, mv.plane_stride, list,
                                                                nblocks, info, crit, mv.f16_unscale);
        break;
    }
}

static void launch_class_any(int b, int cls, double *tiles, int64_t k, const MixedViews &mv, const int2 *list,
                             int64_t count, const int64_t *info, bool critical, bool pair, hipStream_t s)
{
    switch (b) {
    case 128: launch_class<128>(cls, tiles, k, mv, list, count, info, critical, pair, s); break;
    case 256: launch_class<256>(cls, tiles, k, mv, list, count, info, critical, pair, s); break;
    case 384: launch_class<384>(cls, tiles, k, mv, list, count, info, critical, pair, s); break;
    default: launch_class<512>(cls, tiles, k, mv, list, count, info, critical, pair, s); break;
    }
}

// Tiles of column k in a low-precision class receive their FP32 running sum
// of updates: A_ik += Δ_ik (binary64), before the TRSM of step k.
template <int B>
__global__ __launch_bounds__(256) void delta_flush_kernel(double *__restrict__ tiles, const float *__restrict__ delta,
                                                          const uint8_t *__restrict__ map, int64_t k,
                                                          const int64_t *__restrict__ info)
{
    if (*info != 0) return;
    const int64_t i = k + 1 + blockIdx.x;
    if (map[tile_index(i, k)] == C64) return;
    const int64_t off = tile_offset(i, k, B);
    constexpr int64_t CH = (int64_t)B * B / 64;  // elements per chunk (blockIdx.y of 64)
    const int64_t e0 = off + (int64_t)blockIdx.y * CH;
    for (int64_t e = threadIdx.x; e < CH; e += 256) tiles[e0 + e] += (double)delta[e0 + e];
}

static void launch_delta_flush(const Work &w, int64_t k, hipStream_t s)
{
    const int64_t m = w.nt - k - 1;
    if (m <= 0 || k == 0) return;
    dim3 grid((unsigned)m, 64);
    switch (w.b) {
    case 128: delta_flush_kernel<128><<<grid, 256, 0, s>>>(w.tiles, w.mv.delta, w.mv.map, k, w.info); break;
    case 256: delta_flush_kernel<256><<<grid, 256, 0, s>>>(w.tiles, w.mv.delta, w.mv.map, k, w.info); break;
    case 384: delta_flush_kernel<384><<<grid, 256, 0, s>>>(w.tiles, w.mv.delta, w.mv.map, k, w.info); break;
    default: delta_flush_kernel<512><<<grid, 256, 0, s>>>(w.tiles, w.mv.delta, w.mv.map, k, w.info); break;
    }
}

static void launch_panel_convert(const Work &w, int64_t k, const MixedViews &mv, hipStream_t s)
{
    const int64_t m = w.nt - k - 1;
    if (m <= 0) return;
    const int par = (int)(k & 1);
    dim3 grid((unsigned)m, (unsigned)((w.b / 64) * (w.b / 64)));
    float *p32 = mv.p32[par];
    uint16_t *pl = mv.planes[par];
    const float f16s = (float)mv.f16_scale;
    switch (w.b) {
    case 128: panel_convert_kernel<128><<<grid, 256, 0, s>>>(w.tiles, k, p32, pl, mv.plane_stride, mv.np, f16s, w.info); break;
    case 256: panel_convert_kernel<256><<<grid, 256, 0, s>>>(w.tiles, k, p32, pl, mv.plane_stride, mv.np, f16s, w.info); break;
    case 384: panel_convert_kernel<384><<<grid, 256, 0, s>>>(w.tiles, k, p32, pl, mv.plane_stride, mv.np, f16s, w.info); break;
    default: panel_convert_kernel<512><<<grid, 256, 0, s>>>(w.tiles, k, p32, pl, mv.plane_stride, mv.np, f16s, w.info); break;
    }
}

// Device bytes of the mixed-precision side buffers for nt tiles of size b:
// the FP32 running sums, panel copies (two parities; FP32, three bfloat16 or
// two binary16 parts), the tile lists and the precision map.
size_t mixed_extra_bytes(int64_t nt, int b, int precision)
{
    if (precision == GL_FP64) return 0;
    const size_t slot = (size_t)nt * b * b;
    const size_t parts = (precision == GL_MIXED_FP16) ? 2 : 3;
    size_t panel = (precision == GL_MIXED_FP32) ? 2 * slot * sizeof(float) : 2 * parts * slot * sizeof(uint16_t);
    const size_t tc = (size_t)tile_count(nt);
    return tc * b * b * sizeof(float) + panel + tc * sizeof(int2) + ((tc + 255) / 256) * 256 + 1024;
}

void mixed_views(Work &w)
{
    MixedViews &mv = w.mv;
    mv = MixedViews{};
    if (w.precision == GL_FP64 || !w.mix) return;
    const size_t slot = (size_t)w.nt * w.b * w.b;
    char *p = static_cast<char *>(w.mix);
    mv.delta = reinterpret_cast<float *>(p);  // one FP32 b×b block per tile, packed like the tiles
    p += (size_t)tile_count(w.nt) * w.b * w.b * sizeof(float);
    if (w.precision == GL_MIXED_FP32) {
        mv.p32[0] = reinterpret_cast<float *>(p);
        mv.p32[1] = mv.p32[0] + slot;
        p += 2 * slot * sizeof(float);
        mv.np = 0;
    } else {
        const int parts = (w.precision == GL_MIXED_FP16) ? 2 : 3;
        mv.planes[0] = reinterpret_cast<uint16_t *>(p);
        mv.planes[1] = mv.planes[0] + parts * slot;
        mv.plane_stride = (int64_t)slot;
        mv.np = parts;
        p += 2 * parts * slot * sizeof(uint16_t);
    }
    const size_t tc = (size_t)tile_count(w.nt);
    mv.lists = reinterpret_cast<int2 *>(p);
    p += tc * sizeof(int2);
    mv.map = reinterpret_cast<uint8_t *>(p);
    p += ((tc + 255) / 256) * 256;
    mv.thr = reinterpret_cast<double *>(p);  // 4 doubles in the 1024-byte tail
}

// Classify the tiles on the device, bring the map to the host, build the
// per-class tile lists in column order and upload them.
static int build_lists(Work &w, const gl_opts &o, hipStream_t s, MixedPlan &plan)
{
    const int64_t nt = w.nt;
    const int64_t tc = tile_count(nt);
    const int mode = w.precision;
    classify_kernel<<<(unsigned)ceil_div(tc, 256), 256, 0, s>>>(w.norm2, nt, o.band, mode, w.mv.thr, w.mv.map);
    GL_HIP_TRY(hipGetLastError());
    std::vector<uint8_t> map((size_t)tc);
    GL_HIP_TRY(hipMemcpyAsync(map.data(), w.mv.map, (size_t)tc, hipMemcpyDeviceToHost, s));
    GL_HIP_TRY(hipMemcpyAsync(plan.thr, w.mv.thr, sizeof(plan.thr), hipMemcpyDeviceToHost, s));
    GL_HIP_TRY(hipStreamSynchronize(s));
    plan.start.assign(NCLASS, std::vector<int64_t>(nt + 2, 0));
    std::vector<int2> all;
    all.reserve((size_t)tc);
    for (int c = 0; c < NCLASS; ++c) {
        plan.base[c] = (int64_t)all.size();
        plan.tiles[c] = 0;
        plan.work[c] = 0.0;
        for (int64_t j = 0; j < nt; ++j) {
            plan.start[c][j] = (int64_t)all.size() - plan.base[c];
            for (int64_t i = j; i < nt; ++i)
                if (map[(size_t)tile_index(i, j)] == c) {
                    all.push_back(make_int2((int)i, (int)j));
                    plan.tiles[c] += 1;
                    plan.work[c] += (double)j;  // tile (i, j) receives j trailing updates
                }
        }
        plan.start[c][nt] = (int64_t)all.size() - plan.base[c];
        plan.start[c][nt + 1] = plan.start[c][nt];
    }
    GL_HIP_TRY(hipMemcpyAsync(w.mv.lists, all.data(), all.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    GL_HIP_TRY(hipStreamSynchronize(s));  // `all` is a host temporary
    return GL_OK;
}

// Trailing updates of step k for tile columns [j0, j1] of every class.
// Which classes a launch group covers: every class with panel k alone, only
// the per-step classes (binary64, FP32) with panel k, or those with panel k
// and the split-product classes with panels k-1 and k.
enum { UPD_ALL = 0, UPD_STEP = 1, UPD_PAIR = 2 };

// Timed (when profiling) in the class's phase with its algorithmic flops:
// 2b³ per off-diagonal tile update and b²(b+1) per diagonal one (every
// column's diagonal tile is in the band, so binary64), twice that with two
// panels.
static void class_updates(Lanes &ln, Work &w, int64_t k, int64_t j0, int64_t j1, const MixedPlan &plan,
                          bool critical, int sel, hipStream_t s)
{
    const double b = (double)w.b, b3 = b * b * b;
    for (int c = 0; c < NCLASS; ++c) {
        if (sel == UPD_STEP && paired_class(c)) continue;
        const bool pair = sel == UPD_PAIR && paired_class(c);
        const int64_t a = plan.start[c][j0], e = plan.start[c][j1 + 1];
        if (e <= a) continue;
        const double ndiag = c == C64 ? (double)(j1 - j0 + 1) : 0.0;
        const double flops = (pair ? 2.0 : 1.0) * (2.0 * b3 * ((double)(e - a) - ndiag) + b * b * (b + 1.0) * ndiag);
        timed(ln.prof, GL_PHASE_MIXED_FP64 + c, flops, s, [&] {
            launch_class_any(w.b, c, w.tiles, k, w.mv, w.mv.lists + plan.base[c] + a, e - a, w.info, critical, pair,
                             s);
        });
    }
}

int mixed_factorize(Lanes &ln, Work &w, gl_theta th, const gl_opts &o, hipStream_t s, MixedPlan *plan_out)
{
    launch_gen_tiles(w.tiles, w.x, w.y, w.n, w.b, w.nt, th, geom_of(o), w.norm2, s);
    launch_fill(reinterpret_cast<double *>(w.mv.delta), tile_count(w.nt) * w.b * w.b / 2, 0.0, s);
    // step 0's POTRF first: its pivots set the adaptive thresholds
    launch_potrf(w.tiles, w.b, 0, w.n, w.info, w.logsum, w.dinv_k(0), s);
    thresholds_kernel<<<1, 256, 0, s>>>(w.tiles, w.b, w.n, th.theta1, w.precision, o.accuracy, o.tol_64, o.tol_hi,
                                        o.tol_lo, w.mv.thr);
    if (w.precision == GL_MIXED_FP16) {
        // every |L_ik| <= sqrt(max Σ_ii) = sqrt(max(θ1, 1)) (padding rows have
        // a unit diagonal); scale that bound to at most 2^14, below the
        // binary16 maximum 65504 with room for rounding
        const int e = 14 - (int)std::ceil(0.5 * std::log2(std::max(th.theta1, 1.0)));
        w.mv.f16_scale = std::ldexp(1.0, e);
        w.mv.f16_unscale = (float)std::ldexp(1.0, -2 * e);
    }
    MixedPlan plan;
    int rc = build_lists(w, o, s, plan);
    if (rc != GL_OK) return rc;
    if (plan_out) *plan_out = plan;
    // Every tile binary64 (the thresholds found no tile whose class error
    // stays within the accuracy target): the binary64 schedule, with its
    // two-panel passes, continues after the POTRF of tile 0 done above.
    bool all64 = true;
    for (int c = 1; c < NCLASS; ++c) all64 = all64 && plan.tiles[c] == 0;
    if (all64) return factorize(ln, w, s, true, near_tiles_for(w.b, o.near_tiles), true);
    hipStream_t la = ln.la;
    const bool pairs = w.precision == GL_MIXED_BF16 || w.precision == GL_MIXED_FP16;
    // Split-product tiles per column, for the split column of each pair below.
    std::vector<int64_t> pcol((size_t)w.nt, 0);
    for (int c = 0; c < NCLASS; ++c)
        if (paired_class(c))
            for (int64_t j = 0; j < w.nt; ++j) pcol[(size_t)j] += plan.start[c][j + 1] - plan.start[c][j];
    const double rb = 512.0 / (double)w.b;
    const int64_t near_tiles = o.near_tiles > 0 ? (int64_t)o.near_tiles : (int64_t)(1536.0 * rb * rb * rb);
    int64_t js = w.nt;  // columns >= js take the current pair of panels in one update
    GL_HIP_TRY(hipEventRecord(ln.fork, s));
    GL_HIP_TRY(hipStreamWaitEvent(la, ln.fork, 0));
    GL_HIP_TRY(hipStreamWaitEvent(ln.sv, ln.fork, 0));
    for (int64_t k = 0; k < w.nt; ++k) {
        if (k > 0) launch_potrf(w.tiles, w.b, k, w.n, w.info, w.logsum, w.dinv_k(k), s);
        launch_delta_flush(w, k, s);
        launch_trsm(w.tiles, w.b, w.nt, k, w.dinv_k(k), w.info, s);
        // column k is final: its forward solve runs on the solve stream
        rc = solve_step(ln, w, k, s);
        if (rc != GL_OK) return rc;
        if (k + 1 < w.nt) {
            // Split-product classes take two steps per update of their running
            // sums.  At an even step k the next column gets panel k (the
            // critical path needs it), and so do the nearest columns up to js,
            // about near_tiles split-product tiles: work for the lookahead
            // stream while step k+1's critical path runs.  Columns from js on
            // defer panel k to step k+1, whose launches apply panels k and
            // k+1 together (both parities are held).  So the parity that an
            // even step writes may still be read by the previous step's bulk
            // launch: wait for it first.
            const bool odd = pairs && (k & 1);
            const bool even_wait = pairs && !odd && k > 0;
            if (pairs && !odd) {
                int64_t acc = 0;
                js = k + 2;
                while (js < w.nt && acc < near_tiles) acc += pcol[(size_t)js++];
            }
            if (even_wait) GL_HIP_TRY(hipStreamWaitEvent(s, ln.bulk, 0));
            launch_panel_convert(w, k, w.mv, s);
            GL_HIP_TRY(hipEventRecord(ln.panel, s));
            if (k > 0 && !even_wait) GL_HIP_TRY(hipStreamWaitEvent(s, ln.bulk, 0));
            class_updates(ln, w, k, k + 1, k + 1, plan, true, (odd && k + 1 >= js) ? UPD_PAIR : UPD_ALL, s);
            if (k + 2 < w.nt) {
                GL_HIP_TRY(hipStreamWaitEvent(la, ln.panel, 0));
                if (!pairs) {
                    class_updates(ln, w, k, k + 2, w.nt - 1, plan, false, UPD_ALL, la);
                } else {
                    const int64_t split = std::max(js, k + 2);
                    if (split > k + 2) class_updates(ln, w, k, k + 2, split - 1, plan, false, UPD_ALL, la);
                    if (split < w.nt) class_updates(ln, w, k, split, w.nt - 1, plan, false, odd ? UPD_PAIR : UPD_STEP, la);
                }
                GL_HIP_TRY(hipEventRecord(ln.bulk, la));
            }
        }
    }
    GL_HIP_TRY(hipGetLastError());
    GL_HIP_TRY(hipEventRecord(ln.join, la));
    GL_HIP_TRY(hipStreamWaitEvent(s, ln.join, 0));
    return solve_join(ln, s);
}

}  // namespace gl
