// Spatial reordering of the locations along a Morton (Z-order) curve.
//
// l(θ) does not depend on the order of the locations (a permutation P gives
// P Σ Pᵀ and P Z, with the same determinant and quadratic form), so the
// library may factor the covariance in any order.  Ordering along a Morton
// curve makes each tile a compact patch of the domain, so the covariance of
// two distant tiles is small; the mixed-precision path relies on that.
//
// Keys: coordinates are quantised to 16 bits over their bounding box,
//   q = floor((x - min) / (max - min) · 65535),
// interleaved (x in the even bits) into a 32-bit code, and combined with the
// point index as (code << 32) | index.  The keys are unique, so the sorted
// order — and the permutation — is fully determined (bit-exact) whatever the
// sorting network; a bitonic network over the keys padded to a power of two
// is used.
#include "engine.hpp"

namespace gl {

__global__ void bbox_kernel(const double *__restrict__ x, const double *__restrict__ y, int64_t n,
                            double *__restrict__ box)
{
    // one workgroup; fixed-order reduction of min and max
    __shared__ double s[4][256];
    double a = INFINITY, b = -INFINITY, c = INFINITY, d = -INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        a = fmin(a, x[i]);
        b = fmax(b, x[i]);
        c = fmin(c, y[i]);
        d = fmax(d, y[i]);
    }
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = b;
    s[2][threadIdx.x] = c;
    s[3][threadIdx.x] = d;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) box[threadIdx.x] = s[threadIdx.x][0];
}

__device__ inline uint32_t spread16(uint32_t v)
{
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ inline uint32_t quantize16(double v, double lo, double hi)
{
    const double span = hi - lo;
    if (!(span > 0.0)) return 0u;
    double q = floor((v - lo) / span * 65535.0);
    q = fmin(fmax(q, 0.0), 65535.0);
    return (uint32_t)q;
}

__global__ void morton_keys_kernel(const double *__restrict__ x, const double *__restrict__ y,
                                   int64_t n, int64_t npow2, const double *__restrict__ box,
                                   uint64_t *__restrict__ keys)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npow2) return;
    if (i >= n) {
        keys[i] = ~0ull;
        return;
    }
    const uint32_t qx = quantize16(x[i], box[0], box[1]);
    const uint32_t qy = quantize16(y[i], box[2], box[3]);
    const uint64_t code = (uint64_t)(spread16(qx) | (spread16(qy) << 1));
    keys[i] = (code << 32) | (uint64_t)i;
}

// One compare-exchange stage (k, j) of the bitonic network, ascending overall.
__global__ void bitonic_stage_kernel(uint64_t *__restrict__ keys, int64_t npow2, int64_t k, int64_t j)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npow2) return;
    const int64_t p = i ^ j;
    if (p <= i) return;
    const bool up = (i & k) == 0;
    const uint64_t a = keys[i], b = keys[p];
    if ((a > b) == up) {
        keys[i] = b;
        keys[p] = a;
    }
}

// Gather x, y, z into padded buffers in key order; perm (optional) receives
// the original index of each reordered position.
__global__ void gather_kernel(const uint64_t *__restrict__ keys, int64_t n, int64_t npad,
                              const double *__restrict__ x, const double *__restrict__ y,
                              const double *__restrict__ z, double *__restrict__ xo,
                              double *__restrict__ yo, double *__restrict__ zo,
                              int64_t *__restrict__ perm)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npad) return;
    if (i < n) {
        const int64_t src = (int64_t)(keys[i] & 0xffffffffull);
        if (xo) xo[i] = x[src];
        if (yo) yo[i] = y[src];
        if (zo) zo[i] = z[src];
        if (perm) perm[i] = src;
    } else {
        if (xo) xo[i] = 0.0;
        if (yo) yo[i] = 0.0;
        if (zo) zo[i] = 0.0;
    }
}

int64_t npow2_of(int64_t n)
{
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// keys must hold npow2 + 4 64-bit words (the tail holds the bounding box).
void launch_morton_order(const double *x, const double *y, const double *z, int64_t n, int64_t npad,
                         uint64_t *keys, double *xo, double *yo, double *zo, int64_t *perm,
                         hipStream_t s)
{
    int64_t npow2 = 1;
    while (npow2 < n) npow2 <<= 1;
    double *box = reinterpret_cast<double *>(keys + npow2);
    bbox_kernel<<<1, 256, 0, s>>>(x, y, n, box);
    const unsigned grid = (unsigned)ceil_div(npow2, 256);
    morton_keys_kernel<<<grid, 256, 0, s>>>(x, y, n, npow2, box, keys);
    for (int64_t k = 2; k <= npow2; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1) bitonic_stage_kernel<<<grid, 256, 0, s>>>(keys, npow2, k, j);
    gather_kernel<<<(unsigned)ceil_div(npad, 256), 256, 0, s>>>(keys, n, npad, x, y, z, xo, yo, zo, perm);
}

}  // namespace gl
