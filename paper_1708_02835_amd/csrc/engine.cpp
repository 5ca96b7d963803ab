// C-ABI implementation: contexts, device workspaces, the step schedule of the
// tiled factorisation, and the entry points of geolik.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include <algorithm>

#include "engine.hpp"

int gl_hip_fail(hipError_t e, const char *what)
{
    if (getenv("GEOLIK_VERBOSE")) fprintf(stderr, "geolik: %s failed: %s\n", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? GL_ENOMEM : GL_EHIP;
}

namespace gl {

static void graph_drop(gl_context *ctx);

int pick_tile(int64_t n, int32_t requested)
{
    if (requested == 128 || requested == 256 || requested == 384 || requested == 512) return requested;
    if (n <= 3000) return 128;
    if (n <= 24000) return 256;
    return 512;
}

bool valid_theta(const gl_theta &t)
{
    return t.theta1 > 0.0 && t.theta2 > 0.0 && t.theta3 > 0.0 && t.theta3 <= 50.0 &&
           isfinite(t.theta1) && isfinite(t.theta2);
}

// The mixed modes keep FP32 running sums of updates whose size is of order θ1.
bool valid_theta_for(const gl_theta &t, const gl_opts &o)
{
    return valid_theta(t) && (o.precision == GL_FP64 || t.theta1 <= 1e30);
}

// Sizes of the three device allocations of a workspace.
static void work_sizes(int64_t n, int b, int precision, size_t &tiles, size_t &vec, size_t &mix)
{
    const int64_t nt = ceil_div(n, b);
    const int64_t npad = nt * b;
    tiles = (size_t)tile_count(nt) * (size_t)b * b * sizeof(double);
    // x, y, v | logsum, quad | norm2 | dinv (every diagonal tile) | info + result | Morton keys
    vec = (size_t)(3 * npad + 2 * nt + tile_count(nt) + 64 * npad + 16 + npow2_of(n) + 4) * sizeof(double);
    mix = mixed_extra_bytes(nt, b, precision);
}

size_t work_bytes(int64_t n, int b, int precision)
{
    size_t t, v, m;
    work_sizes(n, b, precision, t, v, m);
    return t + v + m;
}

void Work::release()
{
    if (tiles) hipFree(tiles);
    if (vecs) hipFree(vecs);
    if (mix) hipFree(mix);
    tiles = nullptr;
    vecs = nullptr;
    mix = nullptr;
    tile_cap = vec_cap = mix_cap = 0;
    mv = MixedViews{};
    ++gen;
}

static int grow(void *&p, size_t &cap, size_t need, uint64_t &gen)
{
    if (need <= cap) return GL_OK;
    ++gen;
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
    GL_HIP_TRY(hipMalloc(&p, need));
    cap = need;
    return GL_OK;
}

// Size the workspace for (n, b); reuses the allocations when they are big enough.
int Work::ensure(gl_context *ctx, int64_t n_, int b_, int precision_)
{
    size_t tneed, vneed, mneed;
    work_sizes(n_, b_, precision_, tneed, vneed, mneed);
    const size_t old = bytes();
    const size_t want = (tneed > tile_cap ? tneed : tile_cap) + (vneed > vec_cap ? vneed : vec_cap) +
                        (mneed > mix_cap ? mneed : mix_cap);
    if (want > old && ctx->used.load() - old + want > ctx->budget) return GL_ENOMEM;
    void *tp = tiles;
    int rc = grow(tp, tile_cap, tneed, gen);
    tiles = static_cast<double *>(tp);
    if (rc == GL_OK) rc = grow(vecs, vec_cap, vneed, gen);
    if (rc == GL_OK && mneed) rc = grow(mix, mix_cap, mneed, gen);
    ctx->used += bytes() - old;
    if (rc != GL_OK) return rc;
    set_views(n_, b_, precision_);
    return GL_OK;
}

// Point a workspace at caller-provided device memory of `cap` bytes (binary64
// only): the tiles first, then the vectors.  Nothing is allocated, and
// release() must never be called on such a view.
int Work::bind(void *base, size_t cap, int64_t n_, int b_)
{
    size_t tneed, vneed, mneed;
    work_sizes(n_, b_, GL_FP64, tneed, vneed, mneed);
    tneed = (tneed + 255) & ~(size_t)255;
    if (tneed + vneed > cap) return GL_ENOMEM;
    tiles = static_cast<double *>(base);
    vecs = static_cast<char *>(base) + tneed;
    mix = nullptr;
    tile_cap = tneed;
    vec_cap = vneed;
    mix_cap = 0;
    set_views(n_, b_, GL_FP64);
    return GL_OK;
}

void Work::set_views(int64_t n_, int b_, int precision_)
{
    n = n_;
    b = b_;
    nt = ceil_div(n_, b_);
    npad = nt * b_;
    precision = precision_;
    double *p = static_cast<double *>(vecs);
    x = p;
    y = p + npad;
    v = p + 2 * npad;
    logsum = p + 3 * npad;
    quad = logsum + nt;
    norm2 = quad + nt;
    dinv = norm2 + tile_count(nt);
    info = reinterpret_cast<int64_t *>(dinv + 64 * npad);
    res = reinterpret_cast<DevResult *>(info + 8);
    keys = reinterpret_cast<uint64_t *>(info + 16);
    mixed_views(*this);
}

int Lanes::create()
{
    GL_HIP_TRY(hipStreamCreateWithFlags(&la, hipStreamNonBlocking));
    GL_HIP_TRY(hipStreamCreateWithFlags(&sv, hipStreamNonBlocking));
    GL_HIP_TRY(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    GL_HIP_TRY(hipEventCreateWithFlags(&panel, hipEventDisableTiming));
    GL_HIP_TRY(hipEventCreateWithFlags(&bulk, hipEventDisableTiming));
    GL_HIP_TRY(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    GL_HIP_TRY(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    GL_HIP_TRY(hipEventCreateWithFlags(&solved, hipEventDisableTiming));
    return GL_OK;
}

void Lanes::destroy()
{
    if (la) hipStreamDestroy(la);
    if (sv) hipStreamDestroy(sv);
    for (hipEvent_t e : {fork, panel, bulk, join, ready, solved})
        if (e) (void)hipEventDestroy(e);
    la = sv = nullptr;
    fork = panel = bulk = join = ready = solved = nullptr;
}

hipEvent_t Prof::take()
{
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
        e = pool.back();
        pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// Timing is best effort: a mark whose events could not be created or
// recorded is dropped, the launch itself is unaffected.
void Prof::begin(hipStream_t s, Mark &m)
{
    m.a = take();
    if (m.a && hipEventRecord(m.a, s) != hipSuccess) {
        pool.push_back(m.a);
        m.a = nullptr;
    }
}

void Prof::end(hipStream_t s, Mark &m, int phase, double flops)
{
    if (!m.a) return;
    m.b = take();
    if (!m.b || hipEventRecord(m.b, s) != hipSuccess) {
        pool.push_back(m.a);
        if (m.b) pool.push_back(m.b);
        return;
    }
    m.phase = phase;
    m.flops = flops;
    pending.push_back(m);
}

// Algorithmic flops of the trailing update of step k over tile columns
// jbeg..jend: 2b³ per off-diagonal tile, b²(b+1) per diagonal tile.
static double trailing_flops(int64_t nt, int64_t jbeg, int64_t jend, int b)
{
    double f = 0.0;
    const double b3 = (double)b * b * b;
    for (int64_t j = jbeg; j <= jend; ++j) f += 2.0 * b3 * (double)(nt - j - 1) + (double)b * b * (b + 1);
    return f;
}

// pair: panels k-1 and k in one pass (K = 2b), twice the flops per tile.
static void trailing(Lanes &ln, Work &w, int64_t k, int64_t jbeg, int64_t jend, hipStream_t s, bool critical,
                     bool pair = false)
{
    timed(ln.prof, critical ? GL_PHASE_TRAIL_CRIT : pair ? GL_PHASE_TRAIL_PAIR : GL_PHASE_TRAIL_BULK,
          (pair ? 2.0 : 1.0) * trailing_flops(w.nt, jbeg, jend, w.b), s,
          [&] { launch_trailing(w.tiles, w.b, w.nt, k, jbeg, jend, w.info, critical, pair, s); });
}

// Default: b tiles (512 at b = 512, about 2.6 ms of update; 256 at b = 256).
// Measured: n = 40,000 at b = 256 takes 0.362 s with 256 near tiles against
// 0.385 s with 4,096; at b = 512 and 384 the time is flat within 1 % from 128
// to 1,024 tiles; at b = 128 it does not depend on it.
int64_t near_tiles_for(int b, int32_t requested)
{
    if (requested > 0) return requested;
    return b;
}

// Tiled right-looking Cholesky (Sec. 5.2) with a one-step lookahead, plus the
// forward solve and the per-tile log-det and wᵀw parts when `solve` is set.
//
// Two panels per pass for the far columns: each trailing pass reads and
// writes its C tile once, so applying panels k and k+1 together (K = 2b)
// halves that traffic and the per-block start-up of the update kernel.  At
// an even step k the next column (the critical path) and the nearest columns,
// up to `near` tiles, get panel k alone: the near part keeps the lookahead
// stream busy while step k+1's POTRF and TRSM run.  The columns beyond
// (from js on) defer panel k to step k+1, whose bulk launch applies panels k
// and k+1 in one pass.  Panels stay final in place, so the deferred launch
// reads them from the tiles.  The order of the subtractions differs from the
// one-panel schedule, the set of products does not.
int factorize(Lanes &ln, Work &w, hipStream_t s, bool solve, int64_t near, bool first_done)
{
    hipStream_t la = ln.la;
    GL_HIP_TRY(hipEventRecord(ln.fork, s));
    GL_HIP_TRY(hipStreamWaitEvent(la, ln.fork, 0));
    if (solve) GL_HIP_TRY(hipStreamWaitEvent(ln.sv, ln.fork, 0));
    const double b3 = (double)w.b * w.b * w.b;
    int64_t js = w.nt;  // columns >= js take the current pair of panels in one pass
    for (int64_t k = 0; k < w.nt; ++k) {
        const double below = (double)(w.nt - k - 1);
        if (k > 0 || !first_done)
            timed(ln.prof, GL_PHASE_POTRF, b3 / 3.0, s,
                  [&] { launch_potrf(w.tiles, w.b, k, w.n, w.info, w.logsum, w.dinv_k(k), s); });
        timed(ln.prof, GL_PHASE_TRSM, b3 * below, s,
              [&] { launch_trsm(w.tiles, w.b, w.nt, k, w.dinv_k(k), w.info, s); });
        // Panel k is final here: the bulk update may start.  The forward solve
        // of step k reads only column k, which no later step changes, and
        // owns v: it runs on its own stream, off the critical path.
        if (k + 1 < w.nt) GL_HIP_TRY(hipEventRecord(ln.panel, s));
        if (solve) {
            const int rc = solve_step(ln, w, k, s);
            if (rc != GL_OK) return rc;
        }
        if (k + 1 < w.nt) {
            const bool odd = (k & 1) != 0;
            if (!odd) {
                // column j holds nt - j tiles
                int64_t acc = 0;
                js = k + 2;
                while (js < w.nt && acc < near) acc += w.nt - js++;
            }
            if (k > 0) GL_HIP_TRY(hipStreamWaitEvent(s, ln.bulk, 0));
            trailing(ln, w, k, k + 1, k + 1, s, true, odd && k + 1 >= js);
            if (k + 2 < w.nt) {
                GL_HIP_TRY(hipStreamWaitEvent(la, ln.panel, 0));
                const int64_t split = std::max(js, k + 2);
                if (split > k + 2) trailing(ln, w, k, k + 2, split - 1, la, false);
                if (split < w.nt && odd) trailing(ln, w, k, split, w.nt - 1, la, false, true);
                GL_HIP_TRY(hipEventRecord(ln.bulk, la));
            }
        }
    }
    GL_HIP_TRY(hipGetLastError());
    GL_HIP_TRY(hipEventRecord(ln.join, la));
    GL_HIP_TRY(hipStreamWaitEvent(s, ln.join, 0));
    return solve ? solve_join(ln, s) : GL_OK;
}

int solve_step(Lanes &ln, Work &w, int64_t k, hipStream_t s)
{
    GL_HIP_TRY(hipEventRecord(ln.ready, s));
    GL_HIP_TRY(hipStreamWaitEvent(ln.sv, ln.ready, 0));
    const double below = (double)(w.nt - k - 1);
    timed(ln.prof, GL_PHASE_SOLVE, (double)w.b * w.b, ln.sv,
          [&] { launch_fwd_diag(w.tiles, w.b, k, w.n, w.v, w.quad, w.dinv_k(k), w.info, ln.sv); });
    timed(ln.prof, GL_PHASE_SOLVE, 2.0 * w.b * w.b * below, ln.sv,
          [&] { launch_fwd_update(w.tiles, w.b, w.nt, k, w.v, w.info, ln.sv); });
    return GL_OK;
}

int solve_join(Lanes &ln, hipStream_t s)
{
    GL_HIP_TRY(hipEventRecord(ln.solved, ln.sv));
    GL_HIP_TRY(hipStreamWaitEvent(s, ln.solved, 0));
    return GL_OK;
}

}  // namespace gl

using namespace gl;

extern "C" {

const char *gl_status_string(int status)
{
    switch (status) {
    case GL_OK: return "ok";
    case GL_NOT_SPD: return "covariance matrix is not positive definite";
    case GL_EINVAL: return "invalid argument";
    case GL_ENOMEM: return "out of device memory or HBM budget exceeded";
    case GL_EHIP: return "HIP runtime error";
    case GL_EBUSY: return "request pending";
    case GL_ECANCELED: return "request cancelled";
    case GL_ETIMEDOUT: return "timed out";
    case GL_ENODEV: return "no usable gfx950 device";
    case GL_EVICTED: return "factor released by the request queue's memory admission";
    case GL_E2BIG: return "workspace exceeds the static scratch buffer (GL_SCRATCH_BYTES)";
    default: return "unknown status";
    }
}

void gl_opts_default(gl_opts *o)
{
    if (!o) return;
    o->precision = GL_FP64;
    o->tile = 0;
    o->keep_factor = 0;
    o->band = 2;
    o->reorder = -1;
    o->metric = GL_EUCLIDEAN;
    o->tol_hi = -1.0;
    o->tol_lo = -1.0;
    o->tol_64 = -1.0;
    o->accuracy = -1.0;
    o->ind_tiles = 0;
    o->graph = 0;
    o->near_tiles = 0;
    o->layout = GL_LAYOUT_DENSE;
    o->radius = 6371.0;
}

int32_t gl_pick_tile(int64_t n, int32_t tile)
{
    if (n < 1 || (tile != 0 && tile != 128 && tile != 256 && tile != 384 && tile != 512)) return GL_EINVAL;
    return pick_tile(n, tile);
}

size_t gl_footprint_bytes(int64_t n, int32_t tile, int32_t precision)
{
    if (n < 1) return 0;
    return work_bytes(n, pick_tile(n, tile), precision);
}

int gl_workspace_layout(int64_t n, int32_t tile, int32_t precision, size_t *tiles_h, size_t *vecs_h,
                        size_t *mix_h)
{
    if (n < 1 || (tile != 0 && tile != 128 && tile != 256 && tile != 384 && tile != 512) ||
        precision < GL_FP64 || precision > GL_MIXED_FP16)
        return GL_EINVAL;
    size_t t, v, m;
    work_sizes(n, pick_tile(n, tile), precision, t, v, m);
    if (tiles_h) *tiles_h = t;
    if (vecs_h) *vecs_h = v;
    if (mix_h) *mix_h = m;
    return GL_OK;
}

int gl_context_create(int device, size_t budget, gl_context **out)
{
    if (!out) return GL_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0 || device < 0 || device >= count)
        return GL_ENODEV;
    hipDeviceProp_t prop;
    GL_HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GL_ENODEV;
    GL_HIP_TRY(hipSetDevice(device));
    gl_context *c = new (std::nothrow) gl_context();
    if (!c) return GL_ENOMEM;
    c->device = device;
    size_t freeb = 0, total = 0;
    GL_HIP_TRY(hipMemGetInfo(&freeb, &total));
    c->budget = budget ? budget : (size_t)(0.9 * (double)freeb);
    if (c->lanes.create() != GL_OK ||
        hipHostMalloc(&c->res_h, sizeof(DevResult), hipHostMallocDefault) != hipSuccess ||
        scratch_init(device, &c->scratch) != GL_OK) {
        gl_context_destroy(c);
        return GL_EHIP;
    }
    *out = c;
    return GL_OK;
}

void gl_context_destroy(gl_context *c)
{
    if (!c) return;
    hipSetDevice(c->device);
    serve_stop_queues(c);
    hipDeviceSynchronize();
    c->ws.release();
    if (c->ind_buf) hipFree(c->ind_buf);
    if (c->ind_host) hipHostFree(c->ind_host);
    if (c->ind_done) hipEventDestroy(c->ind_done);
    graph_drop(c);
    if (c->gs) hipStreamDestroy(c->gs);
    for (hipEvent_t e : c->gev)
        if (e) hipEventDestroy(e);
    if (c->theta_h) hipHostFree(c->theta_h);
    if (c->theta_d) hipFree(c->theta_d);
    for (gl_factor *f : c->factors) {
        f->w.release();
        if (f->used) hipEventDestroy(f->used);
        delete f;
    }
    c->factors.clear();
    serve_context_cleanup(c);
    c->lanes.destroy();
    for (hipEvent_t e : c->prof.pool) hipEventDestroy(e);
    for (const Prof::Mark &m : c->prof.pending) {
        hipEventDestroy(m.a);
        hipEventDestroy(m.b);
    }
    if (c->res_h) hipHostFree(c->res_h);
    delete c;
}

int matern_generate(gl_context *ctx, const double *x1, const double *y1, int64_t n1, const double *x2,
                    const double *y2, int64_t n2, gl_theta th, const gl_opts *opts, double *out, int64_t ld,
                    void *stream)
{
    gl_opts o;
    gl_opts_default(&o);
    if (opts) o = *opts;
    if (!ctx || !x1 || !y1 || !out || n1 < 1 || !valid_theta(th) || !valid_metric(o) ||
        (o.layout != GL_LAYOUT_DENSE && o.layout != GL_LAYOUT_LOWER_TILES))
        return GL_EINVAL;
    if (o.layout == GL_LAYOUT_LOWER_TILES) {
        // Σ of set 1 with itself: set 2 absent or the same arrays
        if ((x2 || y2) && (x2 != x1 || y2 != y1 || n2 != n1)) return GL_EINVAL;
        if (o.tile != 0 && o.tile != 128 && o.tile != 256 && o.tile != 384 && o.tile != 512) return GL_EINVAL;
    } else if (!x2 || !y2 || n2 < 1 || ld < n1) {
        return GL_EINVAL;
    }
    GL_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (o.layout == GL_LAYOUT_LOWER_TILES) {
        const int b = pick_tile(n1, o.tile);
        launch_gen_tiles(out, x1, y1, n1, b, ceil_div(n1, b), th, geom_of(o), nullptr, s);
    } else {
        launch_gen_dense(x1, y1, n1, x2, y2, n2, th, geom_of(o), out, ld, s);
    }
    GL_HIP_TRY(hipGetLastError());
    return GL_OK;
}

}  // extern "C"

namespace gl {

// Likelihood evaluation on a prepared workspace whose x, y, v hold the padded
// inputs.  Leaves the factor and w = L⁻¹ Z in the workspace and enqueues the
// copy of the scalar results to out_h (pinned host memory).
int eval_launch(Lanes &ln, Work &w, gl_theta th, const gl_opts &o, hipStream_t s, DevResult *out_h,
                MixedPlan *plan_out)
{
    launch_fill(reinterpret_cast<double *>(w.info), 1, 0.0, s);
    int rc;
    if (o.precision == GL_FP64) {
        timed(ln.prof, GL_PHASE_GEN, 0.0, s,
              [&] { launch_gen_tiles(w.tiles, w.x, w.y, w.n, w.b, w.nt, th, geom_of(o), nullptr, s); });
        rc = factorize(ln, w, s, true, near_tiles_for(w.b, o.near_tiles));
    } else {
        rc = mixed_factorize(ln, w, th, o, s, plan_out);
    }
    if (rc != GL_OK) return rc;
    timed(o.precision == GL_FP64 ? ln.prof : nullptr, GL_PHASE_REDUCE, 0.0, s,
          [&] { launch_final_reduce(w.logsum, w.quad, w.nt, w.n, w.info, w.res, s); });
    GL_HIP_TRY(hipGetLastError());
    GL_HIP_TRY(hipMemcpyAsync(out_h, w.res, sizeof(DevResult), hipMemcpyDeviceToHost, s));
    return GL_OK;
}

bool valid_metric(const gl_opts &o)
{
    if (o.metric == GL_EUCLIDEAN) return true;
    return o.metric == GL_GREAT_CIRCLE && o.radius > 0.0 && isfinite(o.radius);
}

bool valid_opts(const gl_opts &o)
{
    if (!valid_metric(o)) return false;
    if (o.ind_tiles < 0 || (o.ind_tiles > 0 && (o.precision != GL_FP64 || o.keep_factor))) return false;
    if (o.graph < 0 || o.graph > 1) return false;
    if (o.near_tiles < 0) return false;
    if (o.precision < GL_FP64 || o.precision > GL_MIXED_FP16) return false;
    if (o.tile != 0 && o.tile != 128 && o.tile != 256 && o.tile != 384 && o.tile != 512) return false;
    if (o.reorder < -1 || o.reorder > 1) return false;
    if (o.precision != GL_FP64 && o.band < 1) return false;
    if (isnan(o.tol_hi) || isnan(o.tol_lo) || isnan(o.tol_64) || isnan(o.accuracy)) return false;
    return true;
}

void stage_inputs(Work &w, const double *x, const double *y, const double *z, int reorder, hipStream_t s)
{
    if (reorder) {
        launch_morton_order(x, y, z, w.n, w.npad, w.keys, w.x, w.y, w.v, nullptr, s);
    } else {
        launch_copy_pad(x, w.n, w.x, w.npad, 0.0, s);
        launch_copy_pad(y, w.n, w.y, w.npad, 0.0, s);
        launch_copy_pad(z, w.n, w.v, w.npad, 0.0, s);
    }
}

// Mode defaults for negative thresholds: FP32 mode keeps every off-band tile
// in FP32; BF16 mode uses the three-part split above 1e-2, two parts above
// 1e-4 and one part below.
gl_opts resolved_opts(const gl_opts &in)
{
    gl_opts o = in;
    if (o.accuracy < 0) o.accuracy = 1e-4;
    if (o.reorder < 0) o.reorder = (o.precision == GL_FP64) ? 0 : 1;
    return o;
}

// FP64 evaluation through a captured hipGraph of everything after staging:
// fill, Σ(θ) generation with θ read from device memory, the tiled
// factorisation with its lookahead lane, the final reduction.  The graph is
// captured on the first call for a workspace geometry and distance and
// replayed afterwards; the staging copies and θ's upload run outside it, on
// the same internal stream, ordered after the caller's stream.
static void graph_drop(gl_context *ctx)
{
    if (ctx->gexec) hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
}

static int graph_eval(gl_context *ctx, Work &w, const double *x, const double *y, const double *z, gl_theta th,
                      const gl_opts &o, hipStream_t s)
{
    if (!ctx->gs) {
        GL_HIP_TRY(hipStreamCreateWithFlags(&ctx->gs, hipStreamNonBlocking));
        GL_HIP_TRY(hipEventCreateWithFlags(&ctx->gev[0], hipEventDisableTiming));
        GL_HIP_TRY(hipEventCreateWithFlags(&ctx->gev[1], hipEventDisableTiming));
        GL_HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&ctx->theta_h), sizeof(gl_theta), hipHostMallocDefault));
        GL_HIP_TRY(hipMalloc(reinterpret_cast<void **>(&ctx->theta_d), sizeof(gl_theta)));
    }
    hipStream_t g = ctx->gs;
    const Geom geo = geom_of(o);
    GL_HIP_TRY(hipEventRecord(ctx->gev[0], s));
    GL_HIP_TRY(hipStreamWaitEvent(g, ctx->gev[0], 0));
    stage_inputs(w, x, y, z, o.reorder, g);
    *ctx->theta_h = th;  // the previous call synchronised, so the last upload is done
    GL_HIP_TRY(hipMemcpyAsync(ctx->theta_d, ctx->theta_h, sizeof(gl_theta), hipMemcpyHostToDevice, g));
    // The graph holds pointers into the tiles and into the vectors (x, y, v,
    // the per-tile sums, the diagonal-block inverses, info, result), so any
    // reallocation of the workspace invalidates it, even when the tiles stay.
    const int64_t near = near_tiles_for(w.b, o.near_tiles);
    const bool hit = ctx->gexec && ctx->gkey_gen == w.gen && ctx->gkey_n == w.n && ctx->gkey_b == w.b &&
                     ctx->gkey_geo.metric == geo.metric && ctx->gkey_geo.radius == geo.radius &&
                     ctx->gkey_near == near;
    if (!hit) {
        graph_drop(ctx);
        Lanes ln = ctx->lanes;
        ln.prof = nullptr;  // no timing events inside a graph
        GL_HIP_TRY(hipStreamBeginCapture(g, hipStreamCaptureModeThreadLocal));
        launch_fill(reinterpret_cast<double *>(w.info), 1, 0.0, g);
        launch_gen_tiles_dev(w.tiles, w.x, w.y, w.n, w.b, w.nt, ctx->theta_d, geo, g);
        int rc = factorize(ln, w, g, true, near);
        launch_final_reduce(w.logsum, w.quad, w.nt, w.n, w.info, w.res, g);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(g, &graph);
        if (rc != GL_OK || ec != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            (void)hipGetLastError();
            return rc != GL_OK ? rc : GL_EHIP;
        }
        const hipError_t ei = hipGraphInstantiate(&ctx->gexec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            ctx->gexec = nullptr;
            return GL_EHIP;
        }
        ctx->gkey_gen = w.gen;
        ctx->gkey_n = w.n;
        ctx->gkey_b = w.b;
        ctx->gkey_geo = geo;
        ctx->gkey_near = near;
    }
    GL_HIP_TRY(hipGraphLaunch(ctx->gexec, g));
    GL_HIP_TRY(hipMemcpyAsync(ctx->res_h, w.res, sizeof(DevResult), hipMemcpyDeviceToHost, g));
    GL_HIP_TRY(hipEventRecord(ctx->gev[1], g));
    GL_HIP_TRY(hipStreamWaitEvent(s, ctx->gev[1], 0));
    GL_HIP_TRY(hipStreamSynchronize(g));
    return GL_OK;
}

gl_factor *factor_adopt(gl_context *ctx, const Work &w, gl_theta th, const gl_opts &o, const void *queue)
{
    gl_factor *f = new (std::nothrow) gl_factor();
    if (!f) return nullptr;
    if (hipEventCreateWithFlags(&f->used, hipEventDisableTiming) != hipSuccess) {
        delete f;
        return nullptr;
    }
    f->ctx = ctx;
    f->theta = th;
    f->opts = o;
    f->opts.keep_factor = 1;
    f->w = w;
    f->queue = queue;
    std::lock_guard<std::mutex> lk(ctx->mu);
    f->last_use = ++ctx->use_clock;
    ctx->factors.push_back(f);
    return f;
}

size_t kept_bytes(gl_context *ctx, const void *queue)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    size_t t = 0;
    for (const gl_factor *f : ctx->factors)
        if (f->queue == queue && !f->evicted) t += f->w.bytes();
    return t;
}

size_t evict_factors(gl_context *ctx, const void *queue, size_t want)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    size_t freed = 0;
    while (freed < want) {
        gl_factor *lru = nullptr;
        for (gl_factor *f : ctx->factors)
            if (f->queue == queue && !f->evicted && (!lru || f->last_use < lru->last_use)) lru = f;
        if (!lru) break;
        if (lru->used) (void)hipEventSynchronize(lru->used);  // kernels still reading it
        const size_t b = lru->w.bytes();
        ctx->used -= b;
        lru->w.release();
        lru->evicted = true;
        freed += b;
    }
    return freed;
}

void detach_factors(gl_context *ctx, const void *queue)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (gl_factor *f : ctx->factors)
        if (f->queue == queue) f->queue = nullptr;
}

void fill_result(gl_result *res, const DevResult &d, int b)
{
    res->loglik = d.loglik;
    res->logdet = d.logdet;
    res->quad = d.quad;
    res->info = d.info;
    res->status = d.info ? GL_NOT_SPD : GL_OK;
    res->tile = b;
    res->factor = nullptr;
}

}  // namespace gl

extern "C" {

int loglik_eval(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n,
                gl_theta th, const gl_opts *opts, gl_result *res, void *stream)
{
    if (!res) return GL_EINVAL;
    memset(res, 0, sizeof(*res));
    gl_opts o;
    gl_opts_default(&o);
    if (opts) o = *opts;
    if (!ctx || !x || !y || !z || n < 1 || !valid_opts(o) || !valid_theta_for(th, o)) {
        res->status = GL_EINVAL;
        return GL_EINVAL;
    }
    o = resolved_opts(o);
    GL_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (o.ind_tiles > 0) return ind_eval(ctx, x, y, z, n, th, o, res, s);
    const int b = pick_tile(n, o.tile);
    gl_factor *f = nullptr;
    Work *w = &ctx->ws;
    if (o.keep_factor) {
        f = new (std::nothrow) gl_factor();
        if (!f) return res->status = GL_ENOMEM;
        f->ctx = ctx;
        f->theta = th;
        f->opts = o;
        w = &f->w;
    }
    int rc = w->ensure(ctx, n, b, o.precision);
    if (rc == GL_OK && o.graph && o.precision == GL_FP64 && !f) {
        rc = graph_eval(ctx, *w, x, y, z, th, o, s);
    } else if (rc == GL_OK) {
        stage_inputs(*w, x, y, z, o.reorder, s);
        rc = eval_launch(ctx->lanes, *w, th, o, s, ctx->res_h, &ctx->last_plan);
        if (rc == GL_OK && hipStreamSynchronize(s) != hipSuccess) rc = GL_EHIP;
    }
    if (rc != GL_OK) {
        if (f) {
            ctx->used -= f->w.bytes();
            f->w.release();
            delete f;
        }
        res->status = rc;
        return rc;
    }
    fill_result(res, *ctx->res_h, b);
    if (f) {
        if (res->status == GL_OK) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->factors.push_back(f);
            res->factor = f;
        } else {
            ctx->used -= f->w.bytes();
            f->w.release();
            delete f;
        }
    }
    return res->status;
}

int gl_factor_release(gl_context *ctx, gl_factor *f)
{
    if (!ctx || !f || f->ctx != ctx) return GL_EINVAL;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        bool found = false;
        for (size_t i = 0; i < ctx->factors.size(); ++i)
            if (ctx->factors[i] == f) {
                ctx->factors.erase(ctx->factors.begin() + i);
                found = true;
                break;
            }
        if (!found) return GL_EINVAL;
    }
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    ctx->used -= f->w.bytes();
    f->w.release();
    if (f->used) hipEventDestroy(f->used);
    delete f;
    return GL_OK;
}

int gl_factor_shape(const gl_factor *f, int64_t *n, int32_t *tile)
{
    if (!f) return GL_EINVAL;
    if (n) *n = f->w.n;
    if (tile) *tile = f->w.b;
    return GL_OK;
}

int gl_factor_to_dense(gl_context *ctx, gl_factor *f, double *out, int64_t ld, void *stream)
{
    if (!ctx || !f || !out) return GL_EINVAL;
    FactorUse use(ctx, f);
    if (use.status != GL_OK) return use.status;
    if (ld < f->w.n) return GL_EINVAL;
    GL_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_tiles_to_dense(f->w.tiles, f->w.b, f->w.n, out, ld, s);
    GL_HIP_TRY(hipGetLastError());
    use.finish(s);
    return GL_OK;
}

int krige_predict(gl_context *ctx, gl_factor *f, const double *xnew, const double *ynew, int64_t m,
                  double *znew, double *var, void *stream)
{
    if (!ctx || !f || !xnew || !ynew || !znew || m < 1) return GL_EINVAL;
    FactorUse use(ctx, f);
    if (use.status != GL_OK) return use.status;
    GL_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Work &w = f->w;
    const Geom geo = geom_of(f->opts);
    const int64_t nchunk = krige_chunks(w.n);
    // variances: groups of up to 8 chunks of b right-hand sides
    const int64_t chunks = var ? std::min<int64_t>(8, ceil_div(m, w.b)) : 0;
    const size_t st_len = (size_t)chunks * w.npad * w.b;
    double *scratch = nullptr;
    const size_t bytes = ((size_t)w.npad + m * nchunk + st_len + (size_t)chunks * w.npad) * sizeof(double);
    if (hipMallocAsync(reinterpret_cast<void **>(&scratch), bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        return GL_ENOMEM;
    }
    double *xv = scratch;
    double *part = scratch + w.npad;
    double *st = part + m * nchunk;
    double *vpart = st + st_len;
    // X = L⁻ᵀ w: backward substitution over tile rows, last to first
    GL_HIP_TRY(hipMemcpyAsync(xv, w.v, (size_t)w.npad * sizeof(double), hipMemcpyDeviceToDevice, s));
    for (int64_t k = w.nt - 1; k >= 0; --k) {
        launch_bwd_diag(w.tiles, w.b, k, xv, s);
        launch_bwd_update(w.tiles, w.b, k, xv, s);
    }
    launch_krige(w.x, w.y, w.n, xv, f->theta, geo, xnew, ynew, m, part, nchunk, s);
    launch_krige_reduce(part, m, nchunk, znew, s);
    // var_k = θ1 - ||L⁻¹ σ_k||², right-hand sides solved on the matrix cores
    for (int64_t k0 = 0; var && k0 < m; k0 += chunks * w.b) {
        const int64_t mg = std::min<int64_t>(m - k0, chunks * w.b);
        const int64_t cg = ceil_div(mg, w.b);
        launch_gen_rhs(st, w.x, w.y, w.n, w.b, w.nt, xnew + k0, ynew + k0, mg, cg, f->theta, geo, s);
        for (int64_t k = 0; k < w.nt; ++k) {
            launch_mrhs_diag(w.tiles, st, w.b, w.nt, k, w.dinv_k(k), cg, s);
            launch_mrhs_update(w.tiles, st, w.b, w.nt, k, cg, s);
        }
        launch_rhs_variance(st, w.b, w.nt, cg, mg, f->theta.theta1, vpart, var + k0, s);
    }
    GL_HIP_TRY(hipGetLastError());
    GL_HIP_TRY(hipFreeAsync(scratch, s));
    use.finish(s);
    return GL_OK;
}

int krige_cv(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n, gl_theta th,
             const gl_opts *opts, const int32_t *fold_h, int32_t k, double *mse_h, double *pred_out,
             void *stream)
{
    if (!ctx || !x || !y || !z || !fold_h || !mse_h || n < 2 || k < 2 || !valid_theta(th)) return GL_EINVAL;
    gl_opts o;
    gl_opts_default(&o);
    if (opts) o = *opts;
    const bool ind = o.ind_tiles > 0;  // IND kriging keeps no factor object
    o.keep_factor = ind ? 0 : 1;
    if (!valid_opts(o) || !valid_theta_for(th, o) || (ind && o.reorder == 1)) return GL_EINVAL;
    const gl_opts ro = resolved_opts(o);
    // IND: blocks of ind_tiles·b consecutive locations of the whole input
    const int ib = ind ? pick_tile(n, o.tile) : 0;
    const int64_t iblock = ind ? o.ind_tiles * (int64_t)ib : 1;
    const int64_t nblocks = ind ? ceil_div(n, iblock) : 0;
    std::vector<int64_t> kcount(nblocks), mcount(nblocks);
    std::vector<int64_t> count(k, 0);
    for (int64_t i = 0; i < n; ++i) {
        if (fold_h[i] < 0 || fold_h[i] >= k) return GL_EINVAL;
        ++count[fold_h[i]];
    }
    for (int32_t f = 0; f < k; ++f)
        if (count[f] == 0 || count[f] == n) return GL_EINVAL;
    GL_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // scratch: index list (n) | known x, y, z | missing x, y, z, prediction | mse
    double *buf = nullptr;
    const size_t len = (size_t)n + 7 * (size_t)n + 8;
    if (hipMallocAsync(reinterpret_cast<void **>(&buf), len * sizeof(double), s) != hipSuccess) {
        (void)hipGetLastError();
        return GL_ENOMEM;
    }
    int64_t *idx = reinterpret_cast<int64_t *>(buf);
    double *kx = buf + n, *ky = kx + n, *kz = ky + n;
    double *mx = kz + n, *my = mx + n, *mz = my + n, *pred = mz + n, *dmse = pred + n;
    std::vector<int64_t> order(n);
    int status = GL_OK;
    for (int32_t f = 0; f < k; ++f) {
        // known locations first, then the fold's (missing) ones, each in input order
        int64_t a = 0, b = n - count[f];
        for (int64_t i = 0; i < n; ++i) order[fold_h[i] == f ? b++ : a++] = i;
        const int64_t nk = n - count[f], nm = count[f];
        int rc = GL_OK;
        if (hipMemcpyAsync(idx, order.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = GL_EHIP;
        if (rc == GL_OK) {
            launch_gather3(x, y, z, idx, nk, kx, ky, kz, s);
            launch_gather3(x, y, z, idx + nk, nm, mx, my, mz, s);
            gl_factor *fac = nullptr;
            if (ind) {
                std::fill(kcount.begin(), kcount.end(), 0);
                std::fill(mcount.begin(), mcount.end(), 0);
                for (int64_t i = 0; i < n; ++i) ++(fold_h[i] == f ? mcount : kcount)[i / iblock];
                rc = ind_krige(ctx, kx, ky, kz, kcount.data(), mx, my, mcount.data(), nblocks, th, ro, ib, pred, s);
            } else {
                gl_result r;
                rc = loglik_eval(ctx, kx, ky, kz, nk, th, &o, &r, stream);
                if (rc == GL_OK) {
                    fac = static_cast<gl_factor *>(r.factor);
                    rc = krige_predict(ctx, fac, mx, my, nm, pred, nullptr, stream);
                }
            }
            if (rc == GL_OK) {
                if (pred_out) launch_scatter(pred, idx + nk, nm, pred_out, s);
                launch_mse(pred, mz, nm, dmse, s);
                if (hipMemcpyAsync(&mse_h[f], dmse, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    rc = GL_EHIP;
            } else if (rc == GL_NOT_SPD) {
                mse_h[f] = NAN;
            }
            if (fac) gl_factor_release(ctx, fac);
        }
        if (rc < 0) {
            status = rc;
            break;
        }
        if (rc == GL_NOT_SPD) status = GL_NOT_SPD;
    }
    (void)hipFreeAsync(buf, s);
    (void)hipStreamSynchronize(s);
    return status;
}

int synth_generate(gl_context *ctx, const double *x, const double *y, const double *e, int64_t n,
                   gl_theta th, const gl_opts *opts, double *z, int64_t *info_h, void *stream)
{
    if (!ctx || !x || !y || !e || !z || n < 1 || !valid_theta(th)) return GL_EINVAL;
    gl_opts o;
    gl_opts_default(&o);
    if (opts) o = *opts;
    if (!valid_opts(o) || o.precision != GL_FP64) return GL_EINVAL;
    GL_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Work &w = ctx->ws;
    int rc = w.ensure(ctx, n, pick_tile(n, o.tile), GL_FP64);
    if (rc != GL_OK) return rc;
    launch_copy_pad(x, n, w.x, w.npad, 0.0, s);
    launch_copy_pad(y, n, w.y, w.npad, 0.0, s);
    launch_copy_pad(e, n, w.v, w.npad, 0.0, s);
    launch_fill(reinterpret_cast<double *>(w.info), 1, 0.0, s);
    launch_gen_tiles(w.tiles, w.x, w.y, w.n, w.b, w.nt, th, geom_of(o), nullptr, s);
    rc = factorize(ctx->lanes, w, s, false, near_tiles_for(w.b, o.near_tiles));
    if (rc != GL_OK) return rc;
    // z = L e: e is read from v, the padded product goes to the x buffer (no
    // longer needed once the tiles exist), then its first n values to z
    launch_trmv(w.tiles, w.b, w.nt, w.v, w.x, s);
    GL_HIP_TRY(hipMemcpyAsync(z, w.x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    GL_HIP_TRY(hipMemcpyAsync(ctx->res_h, w.info, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GL_HIP_TRY(hipStreamSynchronize(s));
    const int64_t info = *reinterpret_cast<int64_t *>(ctx->res_h);
    if (info_h) *info_h = info;
    return info ? GL_NOT_SPD : GL_OK;
}

int gl_profile_enable(gl_context *ctx, int32_t on)
{
    if (!ctx || on < 0 || on > 2) return GL_EINVAL;
    ctx->lanes.prof = on ? &ctx->prof : nullptr;
    ctx->prof.all = (on == 2);
    return GL_OK;
}

int gl_profile_phases(gl_context *ctx, double *ms_h, double *flops_h, int64_t *launches_h)
{
    if (!ctx) return GL_EINVAL;
    GL_HIP_TRY(hipSetDevice(ctx->device));
    GL_HIP_TRY(hipDeviceSynchronize());
    Prof &p = ctx->prof;
    double ms[GL_NPHASE] = {}, fl[GL_NPHASE] = {};
    int64_t cnt[GL_NPHASE] = {};
    int rc = GL_OK;
    for (const Prof::Mark &m : p.pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, m.a, m.b) != hipSuccess) rc = GL_EHIP;
        ms[m.phase] += t;
        fl[m.phase] += m.flops;
        cnt[m.phase] += 1;
        p.pool.push_back(m.a);
        p.pool.push_back(m.b);
    }
    p.pending.clear();
    for (int i = 0; i < GL_NPHASE; ++i) {
        if (ms_h) ms_h[i] = ms[i];
        if (flops_h) flops_h[i] = fl[i];
        if (launches_h) launches_h[i] = cnt[i];
    }
    return rc;
}

int gl_profile_read(gl_context *ctx, double *ms_h, double *flops_h, int64_t *launches_h)
{
    double ms[GL_NPHASE], fl[GL_NPHASE];
    int64_t cnt[GL_NPHASE];
    const int rc = gl_profile_phases(ctx, ms, fl, cnt);
    if (rc != GL_OK) return rc;
    if (ms_h) *ms_h = ms[GL_PHASE_TRAIL_CRIT] + ms[GL_PHASE_TRAIL_BULK] + ms[GL_PHASE_TRAIL_PAIR];
    if (flops_h) *flops_h = fl[GL_PHASE_TRAIL_CRIT] + fl[GL_PHASE_TRAIL_BULK] + fl[GL_PHASE_TRAIL_PAIR];
    if (launches_h) *launches_h = cnt[GL_PHASE_TRAIL_CRIT] + cnt[GL_PHASE_TRAIL_BULK] + cnt[GL_PHASE_TRAIL_PAIR];
    return GL_OK;
}

int gl_morton_order(gl_context *ctx, const double *x, const double *y, int64_t n, int64_t *perm, void *stream)
{
    if (!ctx || !x || !y || !perm || n < 1 || n > 0xffffffffll) return GL_EINVAL;
    GL_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint64_t *keys = nullptr;
    GL_HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&keys), (size_t)(npow2_of(n) + 4) * sizeof(uint64_t), s));
    launch_morton_order(x, y, nullptr, n, n, keys, nullptr, nullptr, nullptr, perm, s);
    GL_HIP_TRY(hipGetLastError());
    GL_HIP_TRY(hipFreeAsync(keys, s));
    return GL_OK;
}

int gl_precision_stats(gl_context *ctx, int64_t *tiles_h, double *work_h, double *thresholds_h)
{
    if (!ctx) return GL_EINVAL;
    for (int c = 0; c < GL_NCLASS; ++c) {
        if (tiles_h) tiles_h[c] = ctx->last_plan.tiles[c];
        if (work_h) work_h[c] = ctx->last_plan.work[c];
    }
    for (int c = 0; c < 4; ++c)
        if (thresholds_h) thresholds_h[c] = ctx->last_plan.thr[c];
    return GL_OK;
}

int gl_selftest(gl_context *ctx, int32_t which, double *out_h, int64_t cap)
{
    if (!ctx || !out_h || cap < 256 || which < 0 || which > 3) return GL_EINVAL;
    GL_HIP_TRY(hipSetDevice(ctx->device));
    return selftest_mfma(which, out_h, cap);
}

}  // extern "C"
