// Trailing update of the right-looking tile Cholesky (the SYRK and GEMM tasks
// of the tile algorithm, Sec. 5.2): after step k,
//   A_ij -= L_ik L_jkᵀ   for every tile k < j <= i < NT,
// in FP64 on the matrix cores.
//
// One launch covers the tiles of a range of tile columns [jbeg, jbeg+jcount).
// Each workgroup (256 threads, 4 waves in a 2×2 arrangement) computes one
// 128×128 block of one tile with K = b: the 128-row slices of L_ik and L_jk
// are streamed through LDS in 16-column chunks, double-buffered, and every
// wave accumulates a 64×64 block as 4×4 FP64 16x16x4 products, starting from
// the block's current values.
// Upper blocks of diagonal tiles are skipped (only the lower triangle of A_ii
// is ever read).
//
// Workgroups are dispatched round-robin over the 8 XCDs; the logical block
// index is remapped so that each XCD works on a contiguous run of blocks,
// i.e. on whole tiles and on neighbouring tiles of one column, which share
// the L_jk operand in that XCD's L2.
#include "batch.hpp"
#include "common.hpp"
#include "mfma.hpp"

namespace gl {

constexpr int GB = 128;  // output block edge
constexpr int GK = 16;   // k chunk

// Tiles of columns jbeg, jbeg+1, ... in column order; column jbeg + c holds
// rows i = jbeg + c .. nt-1.  Maps a linear index to (i, j).
__device__ inline void trailing_tile(int64_t t, int64_t jbeg, int64_t nt, int64_t &i, int64_t &j)
{
    const int64_t m0 = nt - jbeg;
    const double a = 2.0 * (double)m0 + 1.0;
    int64_t c = (int64_t)((a - sqrt(a * a - 8.0 * (double)t)) * 0.5);
    if (c < 0) c = 0;
    while (c > 0 && c * m0 - c * (c - 1) / 2 > t) --c;
    while ((c + 1) * m0 - (c + 1) * c / 2 <= t) ++c;
    j = jbeg + c;
    i = j + (t - (c * m0 - c * (c - 1) / 2));
}

// One 128×128 block (rb, cb) of C -= A Bᵀ, all three b×b column-major (ld b).
// The accumulators start from the negated C block and accumulate A Bᵀ - C;
// the block is written once at the end, negated back (no read-modify-write
// after the K loop).  Loader lanes 16·c .. 16·c+15 move 256
// contiguous bytes of one column, so the LDS stores are conflict-free; LDS
// rows are padded to 144 doubles so that the two 16-lane halves of an MFMA
// operand read (rows k and k+1) fall in different banks.
constexpr int GP = GB + 16;  // LDS row pitch (doubles)
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

//
// With a second pair of operands (A2t, B2t non-null: PAIR) the K loop runs
// over both, C -= A Bᵀ + A2 B2ᵀ with K = 2b: two panels applied with one read
// and one write of C.
template <int B, bool PAIR = false>
__device__ __forceinline__ void trailing_core(const double *__restrict__ At, const double *__restrict__ Bt,
                                              double *__restrict__ Ct, int rb, int cb,
                                              const double *__restrict__ A2t = nullptr,
                                              const double *__restrict__ B2t = nullptr)
{
    const double *Ap = At + rb * GB;
    const double *Bp = Bt + cb * GB;
    const double *Ap2 = PAIR ? A2t + rb * GB : Ap;
    const double *Bp2 = PAIR ? B2t + cb * GB : Bp;
    double *C = Ct + (int64_t)(cb * GB) * B + rb * GB;

    __shared__ double As[2][GK][GP];
    __shared__ double Bs[2][GK][GP];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lc = tid >> 4;        // chunk column 0..15
    const int le = (tid & 15) * 2;  // rows le + 32 q, le + 32 q + 1 (q = 0..3)

    // the C block's loads go first, so their latency overlaps the staging of
    // the first chunk; the accumulators are negated once both have arrived.
    // C goes through buffer loads and stores: one per-lane offset register
    // and uniform offsets per element, so no 64-bit address of the 64
    // elements stays live across the k loop
    const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(C, (short)0, B * B * 8, 0x00020000);
    const int cvo = ((wn * 64 + mfma_row(lane, 0)) * B + wm * 64 + mfma_col(lane)) * 8;
    d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[a][b][r] = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(crs, cvo, ((b * 16 + 4 * r) * B + a * 16) * 8, 0));
    d2 ra[4], rbv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ra[q] = *reinterpret_cast<const d2 *>(Ap + (int64_t)lc * B + le + 32 * q);
        rbv[q] = *reinterpret_cast<const d2 *>(Bp + (int64_t)lc * B + le + 32 * q);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        *reinterpret_cast<d2 *>(&As[0][lc][le + 32 * q]) = ra[q];
        *reinterpret_cast<d2 *>(&Bs[0][lc][le + 32 * q]) = rbv[q];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = -acc[a][b];
    __syncthreads();

    constexpr int NK1 = B / GK;
    constexpr int NK = PAIR ? 2 * NK1 : NK1;
    for (int kc = 0; kc < NK; ++kc) {
        const int cur = kc & 1;
        if (kc + 1 < NK) {
            const bool second = PAIR && kc + 1 >= NK1;
            const double *An = second ? Ap2 : Ap;
            const double *Bn = second ? Bp2 : Bp;
            const int64_t col = (int64_t)((kc + 1) - (second ? NK1 : 0)) * GK + lc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ra[q] = *reinterpret_cast<const d2 *>(An + col * B + le + 32 * q);
                rbv[q] = *reinterpret_cast<const d2 *>(Bn + col * B + le + 32 * q);
            }
        }
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            double av[4], bv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                av[q] = As[cur][kk + (lane >> 4)][wm * 64 + q * 16 + (lane & 15)];
                bv[q] = Bs[cur][kk + (lane >> 4)][wn * 64 + q * 16 + (lane & 15)];
            }
            // operands swapped: the product is the transpose of the C block, so
            // result row r of lane l is C column, lane % 16 is C row (coalesced)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma_f64(bv[b], av[a], acc[a][b]);
        }
        // keep the staging of the next chunk after this chunk's products: its
        // stores wait for global loads issued at the top of the iteration, and
        // hoisted above the products they would expose that latency
        __builtin_amdgcn_sched_barrier(0);
        if (kc + 1 < NK) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                *reinterpret_cast<d2 *>(&As[cur ^ 1][lc][le + 32 * q]) = ra[q];
                *reinterpret_cast<d2 *>(&Bs[cur ^ 1][lc][le + 32 * q]) = rbv[q];
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, -acc[a][b][r]), crs, cvo,
                                                      ((b * 16 + 4 * r) * B + a * 16) * 8, 0);
}

// One 128×128 block (rb, cb) of the update of tile (i, j) by panel column k
// (PAIR: by panel columns k-1 and k).
template <int B, bool PAIR = false>
__device__ __forceinline__ void trailing_block_body(double *__restrict__ tiles, int64_t k, int64_t i,
                                                    int64_t j, int rb, int cb)
{
    if (PAIR)
        trailing_core<B, true>(tiles + tile_offset(i, k - 1, B), tiles + tile_offset(j, k - 1, B),
                               tiles + tile_offset(i, j, B), rb, cb, tiles + tile_offset(i, k, B),
                               tiles + tile_offset(j, k, B));
    else
        trailing_core<B>(tiles + tile_offset(i, k, B), tiles + tile_offset(j, k, B), tiles + tile_offset(i, j, B),
                         rb, cb);
}

template <int B, bool PAIR = false>
__global__ __launch_bounds__(256, 2) void trailing_f64_kernel(double *__restrict__ tiles, int64_t k,
                                                              int64_t jbeg, int64_t nt,
                                                              int64_t nblocks,
                                                              const int64_t *__restrict__ info,
                                                              int critical,
                                                              const int2 *__restrict__ list)
{
    if (*info != 0) return;
    if (critical) __builtin_amdgcn_s_setprio(3);
    constexpr int SB = B / GB;
    constexpr int SUB = SB * SB;
    const int64_t G = gridDim.x;  // a multiple of 8
    const int64_t g = blockIdx.x;
    const int64_t lid = (g & 7) * (G >> 3) + (g >> 3);
    if (lid >= nblocks) return;
    const int64_t t = lid / SUB;
    const int sub = (int)(lid % SUB);
    int64_t i, j;
    if (list) {
        const int2 ij = list[t];
        i = ij.x;
        j = ij.y;
    } else {
        trailing_tile(t, jbeg, nt, i, j);
    }
    const int rb = sub / SB, cb = sub % SB;
    if (i == j && cb > rb) return;
    trailing_block_body<B, PAIR>(tiles, k, i, j, rb, cb);
}

template <bool PAIR>
static void launch_trailing_t(double *tiles, int b, int64_t nt, int64_t k, int64_t jbeg, int64_t jend,
                              const int64_t *info, bool critical, hipStream_t s)
{
    if (jbeg > jend || jbeg >= nt) return;
    // tiles in columns jbeg..jend, rows j..nt-1
    const int64_t m0 = nt - jbeg;
    const int64_t cols = jend - jbeg + 1;
    const int64_t ntiles = cols * m0 - cols * (cols - 1) / 2;
    const int64_t sub = (int64_t)(b / GB) * (b / GB);
    const int64_t nblocks = ntiles * sub;
    const int64_t grid = ceil_div(nblocks, 8) * 8;
    const int crit = critical ? 1 : 0;
    switch (b) {
    case 128: trailing_f64_kernel<128, PAIR><<<(unsigned)grid, 256, 0, s>>>(tiles, k, jbeg, nt, nblocks, info, crit, nullptr); break;
    case 256: trailing_f64_kernel<256, PAIR><<<(unsigned)grid, 256, 0, s>>>(tiles, k, jbeg, nt, nblocks, info, crit, nullptr); break;
    case 384: trailing_f64_kernel<384, PAIR><<<(unsigned)grid, 256, 0, s>>>(tiles, k, jbeg, nt, nblocks, info, crit, nullptr); break;
    default: trailing_f64_kernel<512, PAIR><<<(unsigned)grid, 256, 0, s>>>(tiles, k, jbeg, nt, nblocks, info, crit, nullptr); break;
    }
}

// pair: apply panel columns k-1 and k together (k >= 1; both final).
void launch_trailing(double *tiles, int b, int64_t nt, int64_t k, int64_t jbeg, int64_t jend,
                     const int64_t *info, bool critical, bool pair, hipStream_t s)
{
    if (pair)
        launch_trailing_t<true>(tiles, b, nt, k, jbeg, jend, info, critical, s);
    else
        launch_trailing_t<false>(tiles, b, nt, k, jbeg, jend, info, critical, s);
}

// Fused trailing updates of many requests, each at its own step k (columns
// k+1 .. nt-1).  The flattened block index is remapped XCD-contiguously.
template <int B>
__global__ __launch_bounds__(256, 2) void trailing_batched_kernel(const BatchReq *__restrict__ d, int count,
                                                                  int64_t nblocks)
{
    constexpr int SB = B / GB;
    constexpr int SUB = SB * SB;
    const int64_t G = gridDim.x;
    const int64_t g = blockIdx.x;
    const int64_t lid = (g & 7) * (G >> 3) + (g >> 3);
    if (lid >= nblocks) return;
    const int r = GL_BATCH_FIND(d, count, lid, o_tr);
    const BatchReq &q = d[r];
    if (*q.info != 0) return;
    const int64_t local = lid - q.o_tr;
    const int64_t t = local / SUB;
    const int sub = (int)(local % SUB);
    int64_t i, j;
    trailing_tile(t, q.k + 1, q.nt, i, j);
    const int rb = sub / SB, cb = sub % SB;
    if (i == j && cb > rb) return;
    trailing_block_body<B>(q.tiles, q.k, i, j, rb, cb);
}

void launch_trailing_batched(int b, const BatchReq *d, int count, int64_t blocks, hipStream_t s)
{
    if (blocks <= 0) return;
    const int64_t grid = ceil_div(blocks, 8) * 8;
    switch (b) {
    case 128: trailing_batched_kernel<128><<<(unsigned)grid, 256, 0, s>>>(d, count, blocks); break;
    case 256: trailing_batched_kernel<256><<<(unsigned)grid, 256, 0, s>>>(d, count, blocks); break;
    case 384: trailing_batched_kernel<384><<<(unsigned)grid, 256, 0, s>>>(d, count, blocks); break;
    default: trailing_batched_kernel<512><<<(unsigned)grid, 256, 0, s>>>(d, count, blocks); break;
    }
}

// Trailing updates of the tiles listed in `list` (count tiles, (i, j) pairs);
// pair: by panel columns k-1 and k in one pass.
template <bool PAIR>
static void launch_trailing_list_t(double *tiles, int b, int64_t k, const int2 *list, int64_t count,
                                   const int64_t *info, bool critical, hipStream_t s)
{
    if (count <= 0) return;
    const int64_t sub = (int64_t)(b / GB) * (b / GB);
    const int64_t nblocks = count * sub;
    const int64_t grid = ceil_div(nblocks, 8) * 8;
    const int crit = critical ? 1 : 0;
    switch (b) {
    case 128: trailing_f64_kernel<128, PAIR><<<(unsigned)grid, 256, 0, s>>>(tiles, k, 0, 0, nblocks, info, crit, list); break;
    case 256: trailing_f64_kernel<256, PAIR><<<(unsigned)grid, 256, 0, s>>>(tiles, k, 0, 0, nblocks, info, crit, list); break;
    case 384: trailing_f64_kernel<384, PAIR><<<(unsigned)grid, 256, 0, s>>>(tiles, k, 0, 0, nblocks, info, crit, list); break;
    default: trailing_f64_kernel<512, PAIR><<<(unsigned)grid, 256, 0, s>>>(tiles, k, 0, 0, nblocks, info, crit, list); break;
    }
}

void launch_trailing_list(double *tiles, int b, int64_t k, const int2 *list, int64_t count,
                          const int64_t *info, bool critical, bool pair, hipStream_t s)
{
    if (pair)
        launch_trailing_list_t<true>(tiles, b, k, list, count, info, critical, s);
    else
        launch_trailing_list_t<false>(tiles, b, k, list, count, info, critical, s);
}

// Many right-hand sides, update after diagonal step k (layout of st as for
// the multi-RHS diagonal solve): S(c, i) -= U(c, k) L_ikᵀ for every chunk c
// and tile row i > k.  Blocks of one tile row i (sharing L_ik) are adjacent.
template <int B>
__global__ __launch_bounds__(256, 2) void mrhs_update_kernel(const double *__restrict__ tiles, double *__restrict__ st,
                                                             int64_t nt, int64_t k, int64_t chunks, int64_t nblocks)
{
    constexpr int SB = B / GB;
    constexpr int SUB = SB * SB;
    const int64_t G = gridDim.x;
    const int64_t g = blockIdx.x;
    const int64_t lid = (g & 7) * (G >> 3) + (g >> 3);
    if (lid >= nblocks) return;
    const int sub = (int)(lid % SUB);
    const int64_t tc = lid / SUB;
    const int64_t c = tc % chunks;
    const int64_t i = k + 1 + tc / chunks;
    const int64_t bb = (int64_t)B * B;
    trailing_core<B>(st + (c * nt + k) * bb, tiles + tile_offset(i, k, B), st + (c * nt + i) * bb, sub / SB,
                     sub % SB);
}

void launch_mrhs_update(const double *tiles, double *st, int b, int64_t nt, int64_t k, int64_t chunks,
                        hipStream_t s)
{
    const int64_t m = nt - k - 1;
    if (m <= 0) return;
    const int64_t nblocks = m * chunks * (b / GB) * (b / GB);
    const int64_t grid = ceil_div(nblocks, 8) * 8;
    switch (b) {
    case 128: mrhs_update_kernel<128><<<(unsigned)grid, 256, 0, s>>>(tiles, st, nt, k, chunks, nblocks); break;
    case 256: mrhs_update_kernel<256><<<(unsigned)grid, 256, 0, s>>>(tiles, st, nt, k, chunks, nblocks); break;
    case 384: mrhs_update_kernel<384><<<(unsigned)grid, 256, 0, s>>>(tiles, st, nt, k, chunks, nblocks); break;
    default: mrhs_update_kernel<512><<<(unsigned)grid, 256, 0, s>>>(tiles, st, nt, k, chunks, nblocks); break;
    }
}

}  // namespace gl
