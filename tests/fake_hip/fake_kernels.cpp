// CPU stand-ins for the library's kernel launchers, for the host-only build
// of the queue scheduler (see hip/hip_runtime.h in this folder).  Test
// infrastructure only.  They compute the likelihood of Σ = θ1·I, the
// near-diagonal limit of Eq. (1): l = -n/2 log 2π - n/2 log θ1 - |Z|²/(2θ1),
// with the same division of work as the real path (generation marks the
// diagonal tiles with θ1, each POTRF contributes rows·log θ1 to log|Σ|, each
// forward diagonal solve the squares of its rows of Z over θ1), so results
// travel through the same buffers, descriptors and result copies.  θ1 > 1000
// makes POTRF report a non-positive pivot (info = first column of the tile).
#include <math.h>

#include "batch.hpp"
#include "engine.hpp"

namespace gl {

static int64_t rows_of(int64_t n, int b, int64_t k) { return std::min<int64_t>(b, n - k * (int64_t)b); }

void launch_gen_tiles(double *tiles, const double *, const double *, int64_t, int b, int64_t nt, gl_theta th, Geom,
                      double *, hipStream_t)
{
    for (int64_t k = 0; k < nt; ++k) tiles[tile_offset(k, k, b)] = th.theta1;
}
void launch_gen_tiles_dev(double *tiles, const double *x, const double *y, int64_t n, int b, int64_t nt,
                          const gl_theta *thp, Geom g, hipStream_t s)
{
    launch_gen_tiles(tiles, x, y, n, b, nt, *thp, g, nullptr, s);
}
void launch_gen_dense(const double *x1, const double *y1, int64_t n1, const double *x2, const double *y2, int64_t n2,
                      gl_theta th, Geom, double *out, int64_t ld, hipStream_t)
{
    for (int64_t j = 0; j < n2; ++j)
        for (int64_t i = 0; i < n1; ++i) out[i + j * ld] = (x1[i] == x2[j] && y1[i] == y2[j]) ? th.theta1 : 0.0;
}
void launch_potrf(double *tiles, int b, int64_t k, int64_t n, int64_t *info, double *logsum, double *, hipStream_t)
{
    const double t1 = tiles[tile_offset(k, k, b)];
    if (*info == 0 && t1 > 1000.0) *info = k * b + 1;
    logsum[k] = (double)rows_of(n, b, k) * log(t1);
}
void launch_trsm(double *, int, int64_t, int64_t, const double *, const int64_t *, hipStream_t) {}
void launch_trailing(double *, int, int64_t, int64_t, int64_t, int64_t, const int64_t *, bool, bool, hipStream_t) {}
void launch_fwd_diag(const double *tiles, int b, int64_t k, int64_t n, double *v, double *quad, const double *,
                     const int64_t *, hipStream_t)
{
    const double t1 = tiles[tile_offset(k, k, b)];
    double q = 0.0;
    for (int64_t r = 0; r < rows_of(n, b, k); ++r) q += v[k * b + r] * v[k * b + r];
    quad[k] = q / t1;
}
void launch_fwd_update(const double *, int, int64_t, int64_t, double *, const int64_t *, hipStream_t) {}
void launch_bwd_diag(const double *, int, int64_t, double *, hipStream_t) {}
void launch_bwd_update(const double *, int, int64_t, double *, hipStream_t) {}
void launch_trmv(const double *, int, int64_t, const double *, double *, hipStream_t) {}
void launch_final_reduce(const double *logsum, const double *quad, int64_t nt, int64_t n, const int64_t *info,
                         DevResult *res, hipStream_t)
{
    double ld = 0.0, q = 0.0;
    for (int64_t k = 0; k < nt; ++k) {
        ld += logsum[k];
        q += quad[k];
    }
    res->info = *info;
    res->logdet = *info ? NAN : ld;
    res->quad = *info ? NAN : q;
    res->loglik = *info ? -INFINITY : -0.5 * q - 0.5 * ld - 0.5 * (double)n * log(2.0 * M_PI);
}
void launch_fill(double *p, int64_t count, double v, hipStream_t)
{
    for (int64_t i = 0; i < count; ++i) p[i] = v;
}
void launch_copy_pad(const double *src, int64_t n, double *dst, int64_t npad, double padv, hipStream_t)
{
    for (int64_t i = 0; i < npad; ++i) dst[i] = i < n ? src[i] : padv;
}
void launch_tiles_to_dense(const double *, int, int64_t n, double *out, int64_t ld, hipStream_t)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) out[i + j * ld] = 0.0;
}
void launch_krige(const double *, const double *, int64_t, const double *, gl_theta, Geom, const double *,
                  const double *, int64_t m, double *part, int64_t nchunk, hipStream_t)
{
    for (int64_t i = 0; i < m * nchunk; ++i) part[i] = 0.0;
}
void launch_krige_reduce(const double *part, int64_t m, int64_t nchunk, double *out, hipStream_t)
{
    for (int64_t k = 0; k < m; ++k) {
        double s = 0.0;
        for (int64_t c = 0; c < nchunk; ++c) s += part[k * nchunk + c];
        out[k] = s;
    }
}
int64_t krige_chunks(int64_t n) { return (n + 4095) / 4096; }
void launch_gen_rhs(double *, const double *, const double *, int64_t, int, int64_t, const double *, const double *,
                    int64_t, int64_t, gl_theta, Geom, hipStream_t) {}
void launch_mrhs_diag(const double *, double *, int, int64_t, int64_t, const double *, int64_t, hipStream_t) {}
void launch_mrhs_update(const double *, double *, int, int64_t, int64_t, int64_t, hipStream_t) {}
void launch_rhs_variance(const double *, int, int64_t, int64_t, int64_t m, double theta1, double *, double *var,
                         hipStream_t)
{
    for (int64_t k = 0; k < m; ++k) var[k] = theta1;
}
void launch_gather3(const double *a, const double *b, const double *c, const int64_t *idx, int64_t m, double *oa,
                    double *ob, double *oc, hipStream_t)
{
    for (int64_t i = 0; i < m; ++i) {
        oa[i] = a[idx[i]];
        ob[i] = b[idx[i]];
        oc[i] = c[idx[i]];
    }
}
void launch_scatter(const double *a, const int64_t *idx, int64_t m, double *out, hipStream_t)
{
    for (int64_t i = 0; i < m; ++i) out[idx[i]] = a[i];
}
void launch_mse(const double *p, const double *q, int64_t m, double *out, hipStream_t)
{
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += (p[i] - q[i]) * (p[i] - q[i]);
    *out = s / (double)m;
}
int64_t npow2_of(int64_t n)
{
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}
void launch_morton_order(const double *x, const double *y, const double *z, int64_t n, int64_t npad, uint64_t *,
                         double *xo, double *yo, double *zo, int64_t *perm, hipStream_t s)
{
    if (xo) {
        launch_copy_pad(x, n, xo, npad, 0.0, s);
        launch_copy_pad(y, n, yo, npad, 0.0, s);
        launch_copy_pad(z, n, zo, npad, 0.0, s);
    }
    if (perm)
        for (int64_t i = 0; i < n; ++i) perm[i] = i;
}
int selftest_mfma(int, double *, int64_t) { return GL_EINVAL; }
int scratch_init(int, void **out)
{
    *out = nullptr;
    return GL_OK;
}

// mixed precision: no side buffer; the factorisation is the FP64 stand-in
size_t mixed_extra_bytes(int64_t, int, int) { return 0; }
void mixed_views(Work &) {}
int mixed_factorize(Lanes &, Work &w, gl_theta th, const gl_opts &, hipStream_t s, MixedPlan *)
{
    launch_gen_tiles(w.tiles, w.x, w.y, w.n, w.b, w.nt, th, Geom{0, 0.0}, nullptr, s);
    for (int64_t k = 0; k < w.nt; ++k) {
        launch_potrf(w.tiles, w.b, k, w.n, w.info, w.logsum, nullptr, s);
        launch_fwd_diag(w.tiles, w.b, k, w.n, w.v, w.quad, nullptr, w.info, s);
    }
    return GL_OK;
}

int ind_eval(gl_context *, const double *, const double *, const double *, int64_t, gl_theta, const gl_opts &,
             gl_result *res, hipStream_t)
{
    return res->status = GL_EINVAL;
}
int ind_krige(gl_context *, const double *, const double *, const double *, const int64_t *, const double *,
              const double *, const int64_t *, int64_t, gl_theta, const gl_opts &, int, double *, hipStream_t)
{
    return GL_EINVAL;
}

// fused multi-request launches
void launch_stage_batched(const BatchReq *d, int count, int64_t, hipStream_t s)
{
    for (int i = 0; i < count; ++i)
        if (d[i].is_new) {
            *d[i].info = 0;
            launch_copy_pad(d[i].sx, d[i].n, d[i].x, d[i].npad, 0.0, s);
            launch_copy_pad(d[i].sy, d[i].n, d[i].y, d[i].npad, 0.0, s);
            launch_copy_pad(d[i].sz, d[i].n, d[i].v, d[i].npad, 0.0, s);
        }
}
void launch_gen_batched(int b, const BatchReq *d, int count, int64_t, bool, hipStream_t s)
{
    for (int i = 0; i < count; ++i)
        if (d[i].is_new) launch_gen_tiles(d[i].tiles, d[i].x, d[i].y, d[i].n, b, d[i].nt, d[i].th, d[i].geo, nullptr, s);
}
void launch_potrf_batched(int b, const BatchReq *d, int count, hipStream_t s)
{
    for (int i = 0; i < count; ++i) launch_potrf(d[i].tiles, b, d[i].k, d[i].n, d[i].info, d[i].logsum, d[i].dinv, s);
}
void launch_fwd_diag_batched(int b, const BatchReq *d, int count, hipStream_t s)
{
    for (int i = 0; i < count; ++i)
        launch_fwd_diag(d[i].tiles, b, d[i].k, d[i].n, d[i].v, d[i].quad, d[i].dinv, d[i].info, s);
}
void launch_trsm_batched(int, const BatchReq *, int, int64_t, hipStream_t) {}
void launch_fwd_update_batched(int, const BatchReq *, int, int64_t, hipStream_t) {}
void launch_trailing_batched(int, const BatchReq *, int, int64_t, hipStream_t) {}
void launch_final_batched(const BatchReq *d, int count, hipStream_t s)
{
    for (int i = 0; i < count; ++i)
        if (d[i].finishing) launch_final_reduce(d[i].logsum, d[i].quad, d[i].nt, d[i].n, d[i].info, d[i].res, s);
}

}  // namespace gl
