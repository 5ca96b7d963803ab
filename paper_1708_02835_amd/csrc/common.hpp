// Shared definitions of the geolik HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geolik.h"

#define GL_HIP_TRY(expr)                                   \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return gl_hip_fail(_e, #expr); \
    } while (0)

int gl_hip_fail(hipError_t e, const char *what);

namespace gl {

// Packed lower-triangular tile storage.  Tile (i, j), i >= j, of an NT×NT tile
// grid is a b×b column-major block; tiles follow each other in row order of
// the lower triangle: (0,0), (1,0), (1,1), (2,0), ...
__host__ __device__ inline int64_t tile_index(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }
__host__ __device__ inline int64_t tile_offset(int64_t i, int64_t j, int b)
{
    return tile_index(i, j) * (int64_t)b * b;
}
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t tile_count(int64_t nt) { return nt * (nt + 1) / 2; }

// Per-evaluation scalars reduced on the device.
struct DevResult {
    double loglik;
    double logdet;
    double quad;
    double pad;
    int64_t info;
    int64_t pad2;
};

// Distance used by Σ(θ): metric 0 = Euclidean in the plane, 1 = great-circle
// on a sphere of the given radius (x = longitude, y = latitude, degrees).
struct Geom {
    int32_t metric;
    double radius;
};
inline Geom geom_of(const gl_opts &o) { return Geom{o.metric, o.radius}; }

// Launchers (one per kernel family); all asynchronous on `s`.
// Matérn generation
void launch_gen_tiles(double *tiles, const double *x, const double *y, int64_t n, int b, int64_t nt,
                      gl_theta th, Geom geo, double *tile_norm2, hipStream_t s);
void launch_gen_tiles_dev(double *tiles, const double *x, const double *y, int64_t n, int b, int64_t nt,
                          const gl_theta *thp, Geom geo, hipStream_t s);
void launch_gen_dense(const double *x1, const double *y1, int64_t n1, const double *x2,
                      const double *y2, int64_t n2, gl_theta th, Geom geo, double *out, int64_t ld,
                      hipStream_t s);
// Cholesky steps (FP64)
// POTRF leaves the inverses of the b/64 diagonal 64×64 blocks of L_kk in dinv
// (64·b doubles, column-major blocks); TRSM and the forward solve of the same
// step read them.
void launch_potrf(double *tiles, int b, int64_t k, int64_t n, int64_t *info, double *diag_logsum,
                  double *dinv, hipStream_t s);
void launch_trsm(double *tiles, int b, int64_t nt, int64_t k, const double *dinv, const int64_t *info,
                 hipStream_t s);
void launch_trailing(double *tiles, int b, int64_t nt, int64_t k, int64_t jbeg, int64_t jend,
                     const int64_t *info, bool critical, bool pair, hipStream_t s);
// Solves and reductions
void launch_fwd_diag(const double *tiles, int b, int64_t k, int64_t n, double *v, double *quad_part,
                     const double *dinv, const int64_t *info, hipStream_t s);
void launch_fwd_update(const double *tiles, int b, int64_t nt, int64_t k, double *v,
                       const int64_t *info, hipStream_t s);
void launch_bwd_diag(const double *tiles, int b, int64_t k, double *v, hipStream_t s);
void launch_bwd_update(const double *tiles, int b, int64_t k, double *v, hipStream_t s);
void launch_trmv(const double *tiles, int b, int64_t nt, const double *e, double *z, hipStream_t s);
void launch_final_reduce(const double *logdet_part, const double *quad_part, int64_t nt, int64_t n,
                         const int64_t *info, DevResult *res, hipStream_t s);
void launch_fill(double *p, int64_t count, double v, hipStream_t s);
void launch_copy_pad(const double *src, int64_t n, double *dst, int64_t npad, double padv,
                     hipStream_t s);
void launch_tiles_to_dense(const double *tiles, int b, int64_t n, double *out, int64_t ld,
                           hipStream_t s);
// Kriging
void launch_krige(const double *x, const double *y, int64_t n, const double *v, gl_theta th, Geom geo,
                  const double *xn, const double *yn, int64_t m, double *part, int64_t nchunk,
                  hipStream_t s);
void launch_krige_reduce(const double *part, int64_t m, int64_t nchunk, double *out, hipStream_t s);
int64_t krige_chunks(int64_t n);
// Diagnostics
int selftest_mfma(int which, double *out_h, int64_t cap);

// Kriging variances (Eq. 4): chunks of b right-hand sides solved together.
void launch_gen_rhs(double *st, const double *x, const double *y, int64_t n, int b, int64_t nt, const double *xn,
                    const double *yn, int64_t m, int64_t chunks, gl_theta th, Geom geo, hipStream_t s);
void launch_mrhs_diag(const double *tiles, double *st, int b, int64_t nt, int64_t k, const double *dinv,
                      int64_t chunks, hipStream_t s);
void launch_mrhs_update(const double *tiles, double *st, int b, int64_t nt, int64_t k, int64_t chunks,
                        hipStream_t s);
void launch_rhs_variance(const double *st, int b, int64_t nt, int64_t chunks, int64_t m, double theta1,
                         double *part, double *var, hipStream_t s);

// Cross-validation helpers.
void launch_gather3(const double *a, const double *b, const double *c, const int64_t *idx, int64_t m, double *oa,
                    double *ob, double *oc, hipStream_t s);
void launch_mse(const double *p, const double *q, int64_t m, double *out, hipStream_t s);
void launch_scatter(const double *a, const int64_t *idx, int64_t m, double *out, hipStream_t s);

}  // namespace gl
