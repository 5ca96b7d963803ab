// Internal host-side structures of the geolik runtime.
#pragma once

#include <atomic>
#include <mutex>
#include <vector>

#include "batch.hpp"
#include "common.hpp"

namespace gl {

// Views into the mixed-precision side buffer of a workspace.
struct MixedViews {
    float *p32[2] = {nullptr, nullptr};          // FP32 panel copies, by parity of k
    uint16_t *planes[2] = {nullptr, nullptr};    // bfloat16 (3) or binary16 (2) part planes, by parity of k
    int64_t plane_stride = 0;                    // elements between the parts of one parity
    int np = 0;                                  // parts written per panel element
    int2 *lists = nullptr;                       // per-class tile lists (device)
    uint8_t *map = nullptr;                      // per-tile precision class (device)
    double *thr = nullptr;                       // ρ and the effective thresholds (device, 4 doubles)
    float *delta = nullptr;                      // FP32 running sums of low-precision updates, per tile
    double f16_scale = 0.0;                      // FP16 mode: power of two applied to the panel parts
    float f16_unscale = 1.0f;                    // 1 / f16_scale², applied to the products
};

// Host-side plan of one mixed evaluation: per class, the offset of its list
// and, per tile column j, the list position where column j starts.
struct MixedPlan {
    int64_t base[GL_NCLASS] = {};
    int64_t tiles[GL_NCLASS] = {};
    double work[GL_NCLASS] = {};   // Σ over tiles of the number of trailing updates they receive
    double thr[4] = {0, 0, 0, 0};  // ρ, tol_64, tol_hi, tol_lo as used
    std::vector<std::vector<int64_t>> start;
};

// Device buffers of one likelihood evaluation (or of one kept factor).
struct Work {
    // geometry
    int64_t n = 0, nt = 0, npad = 0;
    int b = 0;
    int precision = GL_FP64;
    // allocations
    double *tiles = nullptr;  // packed lower tiles, binary64
    void *vecs = nullptr;
    void *mix = nullptr;  // mixed-precision side buffer
    size_t tile_cap = 0, vec_cap = 0, mix_cap = 0;
    uint64_t gen = 0;  // bumped whenever an allocation is replaced or released
    // views into vecs
    double *x = nullptr, *y = nullptr;  // padded locations
    double *v = nullptr;                // Z on entry, w = L⁻¹ Z after the evaluation
    double *logsum = nullptr;           // per diagonal tile: 2 Σ log L_rr
    double *quad = nullptr;             // per tile: Σ w_r²
    double *norm2 = nullptr;            // per tile: ||Σ_ij||_F² (mixed precision)
    double *dinv = nullptr;             // inverses of the 64×64 diagonal blocks of every L_kk:
                                        // 64·b doubles per diagonal tile, kept with the factor
    int64_t *info = nullptr;
    DevResult *res = nullptr;
    uint64_t *keys = nullptr;           // Morton sort keys (+ bounding box)
    MixedViews mv;
    int ensure(gl_context *ctx, int64_t n, int b, int precision);
    int bind(void *base, size_t cap, int64_t n, int b);
    void set_views(int64_t n, int b, int precision);
    size_t bytes() const { return tile_cap + vec_cap + mix_cap; }
    double *dinv_k(int64_t k) const { return dinv + k * 64 * (int64_t)b; }
    void release();
};

// Optional kernel timing of the binary64 evaluations: HIP events around
// launches, summed per phase (GL_PHASE_* of geolik.h) when read.
struct Prof {
    struct Mark {
        hipEvent_t a = nullptr, b = nullptr;
        int phase = 0;
        double flops = 0.0;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Mark> pending;  // in launch order
    bool all = false;           // every phase; otherwise the trailing updates only
    bool wants(int phase) const
    {
        return all || phase == GL_PHASE_TRAIL_CRIT || phase == GL_PHASE_TRAIL_BULK || phase == GL_PHASE_TRAIL_PAIR ||
               phase >= GL_PHASE_MIXED_FP64;
    }
    hipEvent_t take();
    void begin(hipStream_t s, Mark &m);
    void end(hipStream_t s, Mark &m, int phase, double flops);
};

// Runs launch() on s, bracketed by timing events when phase is profiled.
template <class F>
void timed(Prof *prof, int phase, double flops, hipStream_t s, F &&launch)
{
    if (!prof || !prof->wants(phase)) {
        launch();
        return;
    }
    Prof::Mark m;
    prof->begin(s, m);
    launch();
    prof->end(s, m, phase, flops);
}

// Side stream and events of one evaluation's step schedule (lookahead).
struct Lanes {
    Prof *prof = nullptr;
    hipStream_t la = nullptr;  // bulk trailing updates (lookahead)
    hipStream_t sv = nullptr;  // forward solve, off the critical path
    hipEvent_t fork = nullptr, panel = nullptr, bulk = nullptr, join = nullptr;
    hipEvent_t ready = nullptr, solved = nullptr;  // column k final (for sv); sv drained
    int create();
    void destroy();
};

int pick_tile(int64_t n, int32_t requested);
bool valid_theta(const gl_theta &t);
bool valid_theta_for(const gl_theta &t, const gl_opts &o);
size_t work_bytes(int64_t n, int b, int precision);
// first_done: the POTRF of tile 0 has already run (logsum[0], dinv of step 0).
int factorize(Lanes &ln, Work &w, hipStream_t s, bool solve, int64_t near, bool first_done = false);
// Forward solve of step k (diagonal block and the update of the rows below)
// on ln.sv once the work queued on s so far (column k final) is done; the
// caller has made ln.sv wait for the inputs.  solve_join makes s wait for
// every solve step queued.
int solve_step(Lanes &ln, Work &w, int64_t k, hipStream_t s);
int solve_join(Lanes &ln, hipStream_t s);
// Tiles updated one panel at a time at even steps (gl_opts.near_tiles; 0:
// b tiles, about 2.6 ms of binary64 update at tile 512).
int64_t near_tiles_for(int b, int32_t requested);
// Enqueue a whole evaluation on s (inputs already in w.x, w.y, w.v) and the
// copy of its scalar results to out_h; does not wait.
int eval_launch(Lanes &ln, Work &w, gl_theta th, const gl_opts &o, hipStream_t s, DevResult *out_h,
                MixedPlan *plan_out = nullptr);
// Copy n inputs into the padded workspace vectors, in Morton order when
// `reorder` is set.
void stage_inputs(Work &w, const double *x, const double *y, const double *z, int reorder, hipStream_t s);
gl_opts resolved_opts(const gl_opts &in);
bool valid_opts(const gl_opts &o);
bool valid_metric(const gl_opts &o);

// mixed precision (mixed.hip)
size_t mixed_extra_bytes(int64_t nt, int b, int precision);
void mixed_views(Work &w);
int mixed_factorize(Lanes &ln, Work &w, gl_theta th, const gl_opts &o, hipStream_t s, MixedPlan *plan_out);
void launch_trailing_list(double *tiles, int b, int64_t k, const int2 *list, int64_t count,
                          const int64_t *info, bool critical, bool pair, hipStream_t s);
// Morton reordering (reorder.hip); keys holds npow2(n) + 4 words
int64_t npow2_of(int64_t n);
void launch_morton_order(const double *x, const double *y, const double *z, int64_t n, int64_t npad,
                         uint64_t *keys, double *xo, double *yo, double *zo, int64_t *perm,
                         hipStream_t s);

// serving (serve.cpp)
struct ServeState;
void serve_context_cleanup(gl_context *ctx);
void serve_stop_queues(gl_context *ctx);  // destroys the context's live queues

void fill_result(gl_result *res, const DevResult &d, int b);

// Device address of the static workspace of loglik_eval_noalloc on `device`
// (noalloc.hip), looked up once per device; the device must be current.
int scratch_init(int device, void **out);

// Factors kept by the request queue (engine.cpp).  factor_adopt takes over
// the device memory of w (a finished evaluation) as a new registered factor
// that `queue` may evict; kept_bytes sums the live ones of a queue;
// evict_factors releases them, least recently used first, until at least
// `want` bytes are free or none is left, and returns the bytes released;
// detach_factors makes a queue's factors permanent (the queue is going away).
gl_factor *factor_adopt(gl_context *ctx, const Work &w, gl_theta th, const gl_opts &o, const void *queue);
size_t kept_bytes(gl_context *ctx, const void *queue);
size_t evict_factors(gl_context *ctx, const void *queue, size_t want);
void detach_factors(gl_context *ctx, const void *queue);

// Independent-blocks approximation (ind.cpp); o resolved and validated.
int ind_eval(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n, gl_theta th,
             const gl_opts &o, gl_result *res, hipStream_t s);
// Kriging under the IND approximation of the covariance of all locations:
// nblocks blocks, block B holding kcount[B] observed locations (consecutive in
// x, y, z) and mcount[B] held-out ones (consecutive in xnew, ynew); each
// held-out value is predicted from its block's observed values (0 when there
// are none).  b: tile size of the block factorisations (o.ind_tiles tiles per
// block at most).  GL_NOT_SPD when a block's factorisation fails.
int ind_krige(gl_context *ctx, const double *x, const double *y, const double *z, const int64_t *kcount,
              const double *xnew, const double *ynew, const int64_t *mcount, int64_t nblocks, gl_theta th,
              const gl_opts &o, int b, double *znew, hipStream_t s);

}  // namespace gl

struct gl_factor {
    gl_context *ctx = nullptr;
    gl_theta theta{};
    gl_opts opts{};  // options of the evaluation (distance, precision, order)
    gl::Work w;
    // Factors kept through the request queue: when the queue's admission needs
    // room it releases their device memory, least recently used first; the
    // handle stays valid (calls on it return GL_EVICTED) until
    // gl_factor_release.  All four fields are guarded by ctx->mu.
    const void *queue = nullptr;  // the queue that may evict it (NULL: never)
    uint64_t last_use = 0;        // ctx->use_clock at creation or the last kriging call
    hipEvent_t used = nullptr;    // recorded after the last kernels that read it
    bool evicted = false;
};

struct gl_context {
    int device = 0;
    size_t budget = 0;
    std::atomic<size_t> used{0};
    gl::Work ws;  // reused by evaluations that do not keep their factor
    gl::Lanes lanes;  // step-schedule side stream of the direct calls
    gl::Prof prof;
    gl::MixedPlan last_plan;  // precision map summary of the last mixed evaluation
    gl::DevResult *res_h = nullptr;  // pinned host copy of the last result
    std::mutex mu;                   // guards factors and datasets
    std::vector<gl_factor *> factors;
    uint64_t use_clock = 0;          // orders factor uses for least-recently-used release
    gl::ServeState *serve = nullptr;
    void *ind_buf = nullptr;  // workspace of the independent-blocks evaluations
    size_t ind_cap = 0;
    gl::BatchReq *ind_host = nullptr;  // pinned step descriptors of the IND launches
    size_t ind_host_cap = 0;           // entries
    hipEvent_t ind_done = nullptr;     // recorded after the last IND step's launches
    // replayed evaluation graph (gl_opts.graph): one entry, keyed by the
    // workspace geometry and the distance
    hipStream_t gs = nullptr;        // stream the graph is captured on and replayed on
    hipEvent_t gev[2] = {nullptr, nullptr};
    hipGraphExec_t gexec = nullptr;
    uint64_t gkey_gen = 0;  // ws.gen at capture: the graph holds pointers into every allocation
    int64_t gkey_n = 0;
    int gkey_b = 0;
    gl::Geom gkey_geo{0, 0.0};
    int64_t gkey_near = 0;
    gl_theta *theta_h = nullptr;  // pinned
    gl_theta *theta_d = nullptr;  // device
    void *scratch = nullptr;      // this device's static workspace of loglik_eval_noalloc
};

namespace gl {

// Held by a direct call while it reads a factor: keeps the queue from
// evicting it, checks that it is one of ctx's live factors and records its
// use.  finish(s) records, on the stream of the call's last kernel, the event
// an eviction waits for.
struct FactorUse {
    std::unique_lock<std::mutex> lk;
    gl_factor *f;
    int status = GL_OK;
    FactorUse(gl_context *ctx, gl_factor *fac) : lk(ctx->mu), f(fac)
    {
        bool found = false;
        for (gl_factor *g : ctx->factors) found = found || g == fac;
        if (!found || fac->ctx != ctx) {
            status = GL_EINVAL;
        } else if (fac->evicted) {
            status = GL_EVICTED;
        } else {
            fac->last_use = ++ctx->use_clock;
        }
    }
    void finish(hipStream_t s)
    {
        if (status == GL_OK && f->used) (void)hipEventRecord(f->used, s);
    }
};

}  // namespace gl
