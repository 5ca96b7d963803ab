// Request queue for many concurrent likelihood clients (the optimiser callbacks
// of Sec. 6.3, each asking for l(θ) at a new θ).
//
// A scheduler thread serves requests in two ways.
//
// Continuous batching (FP64 requests with n <= small_n): admitted requests
// join a resident set; every scheduler tick advances each resident request by
// one step of its tiled factorisation through one fused launch per kernel
// (staging and Σ generation for newcomers, POTRF, forward diagonal solve,
// TRSM, forward update, trailing update, final reduction for those whose last
// step it is).  A launch covers all residents of a cohort, each at its own
// step, so requests that arrive while others are on the device join at the
// next tick and leave when done.  Residents are spread over two cohorts with
// their own streams; each cohort may have two ticks in flight.  Each request runs the
// same per-request code as a single evaluation with tile 256, so its result
// does not depend on the batch it rides in.
//
// Other requests use device slots (a stream, a lookahead lane, a workspace
// and a pinned result buffer each) and run their whole evaluation on the
// slot's stream.
//
// Admission is in arrival order, while the resident count stays within
// max_inflight and the workspaces held stay within the HBM budget.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "batch.hpp"
#include "engine.hpp"

namespace gl {

struct Dataset {
    uint64_t id = 0;
    int64_t n = 0;
    double *buf = nullptr;  // x | y | z, n each
    std::atomic<int> refs{0};
    std::atomic<bool> dropped{false};
    std::atomic<bool> freed{false};
    void free_once()
    {
        if (!freed.exchange(true)) {
            if (buf) hipFree(buf);
            buf = nullptr;
        }
    }
};

struct ServeState {
    std::mutex mu;
    std::map<uint64_t, Dataset *> sets;
    std::vector<Dataset *> graveyard;  // dropped datasets, deleted with the context
    std::vector<lq_queue *> queues;
    uint64_t next = 1;
};

static ServeState *serve_state(gl_context *ctx)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->serve) ctx->serve = new ServeState();
    return ctx->serve;
}

void serve_stop_queues(gl_context *ctx)
{
    ServeState *st = ctx->serve;
    if (!st) return;
    std::vector<lq_queue *> qs;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        qs = st->queues;
    }
    for (lq_queue *q : qs) lq_destroy(q);  // each removes itself from st->queues
}

void serve_context_cleanup(gl_context *ctx)
{
    ServeState *st = ctx->serve;
    if (!st) return;
    for (auto &kv : st->sets) {
        kv.second->free_once();
        delete kv.second;
    }
    for (Dataset *d : st->graveyard) {
        d->free_once();
        delete d;
    }
    delete st;
    ctx->serve = nullptr;
}

}  // namespace gl

using namespace gl;

namespace {

enum ReqState { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Request {
    uint64_t ticket = 0;
    Dataset *ds = nullptr;
    gl_theta th{};
    gl_opts o{};
    int state = QUEUED;
    gl_result res{};
};

struct Slot {
    hipStream_t s = nullptr;
    Lanes ln;
    Work w;
    DevResult *res_h = nullptr;
    hipEvent_t done = nullptr;
    Request *req = nullptr;
};

constexpr int TICK_B = 256;     // tile size of the batched engine
constexpr int TICK_RING = 4;    // descriptor buffers
constexpr int TICK_DEPTH = 2;   // ticks in flight
constexpr int TICK_MAX = 64;    // residents per tick

struct Resident {
    Request *req = nullptr;
    Work *w = nullptr;
    int64_t k = 0;
    bool is_new = true;
};

struct TickBuf {
    BatchReq *host = nullptr;  // pinned
    BatchReq *dev = nullptr;
    DevResult *res_h = nullptr;  // pinned, one per finishing request
    hipEvent_t start = nullptr;  // recorded before the tick's first command (timing)
    hipEvent_t done = nullptr;   // recorded after its last (timing)
    bool busy = false;
    std::vector<Resident> finishing;
};

// Residents are split into cohorts that tick independently on their own
// streams, so one cohort's short, narrow launches (POTRF, TRSM, solves)
// overlap another cohort's wide trailing update.
constexpr int NCOHORT = 2;

struct Cohort {
    hipStream_t s = nullptr;
    std::vector<Resident> residents;
    TickBuf ring[TICK_RING];
    int ring_next = 0;
    std::deque<int> ticks;  // ring indices in flight, oldest first
    hipEvent_t last_done = nullptr;  // done event of the last retired tick (gap timing)
};

}  // namespace

struct lq_queue {
    gl_context *ctx = nullptr;
    lq_config cfg{};
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<Slot> slots;
    // continuous batching
    Cohort co[NCOHORT];
    std::vector<Work *> pool;  // idle workspaces of the batched engine
    int inflight = 0, peak_inflight = 0;
    size_t peak_bytes = 0;
    uint64_t completed = 0, fused = 0;
    // tick overhead: host time spent building and enqueuing ticks, device time
    // of the ticks (first to last command) and device idle time between
    // consecutive ticks of a cohort
    uint64_t ticks = 0;
    double host_us = 0.0, device_ms = 0.0, gap_ms = 0.0;
    std::thread thr;
};

namespace {

void finish(lq_queue *q, Request *r, int status)
{
    r->res.status = status;
    r->state = DONE;
    Dataset *d = r->ds;
    r->ds = nullptr;
    if (d && d->refs.fetch_sub(1) == 1 && d->dropped.load()) d->free_once();
    q->cv_done.notify_all();
}

size_t slot_bytes(const Slot &sl) { return sl.w.bytes(); }

size_t held_bytes(const lq_queue *q)
{
    size_t t = kept_bytes(q->ctx, q);  // factors handed out and not yet evicted
    for (const Slot &sl : q->slots) t += slot_bytes(sl);
    for (const Work *w : q->pool) t += w->bytes();
    for (const Cohort &c : q->co) {
        for (const Resident &r : c.residents) t += r.w->bytes();
        for (const TickBuf &tb : c.ring)
            for (const Resident &r : tb.finishing) t += r.w->bytes();
    }
    return t;
}

bool batch_eligible(const lq_queue *q, const Request *r)
{
    return q->cfg.batch_small && r->o.precision == GL_FP64 && r->o.reorder == 0 &&
           (r->o.tile == 0 || r->o.tile == TICK_B) && r->ds->n <= q->cfg.small_n;
}

// A workspace for n points: the smallest pooled one that is large enough,
// else a new one (growing a pooled workspace would free memory, which waits
// for the device; smaller pooled workspaces stay for smaller requests).
int take_work(lq_queue *q, int64_t n, Work *&out)
{
    const size_t need = work_bytes(n, TICK_B, GL_FP64);
    size_t pick = q->pool.size();
    for (size_t i = 0; i < q->pool.size(); ++i)
        if (q->pool[i]->bytes() >= need && (pick == q->pool.size() || q->pool[i]->bytes() < q->pool[pick]->bytes()))
            pick = i;
    Work *w;
    if (pick < q->pool.size()) {
        w = q->pool[pick];
        q->pool.erase(q->pool.begin() + pick);
    } else {
        w = new Work();
    }
    const int rc = w->ensure(q->ctx, n, TICK_B, GL_FP64);
    if (rc != GL_OK) {
        q->ctx->used -= w->bytes();
        w->release();
        delete w;
        return rc;
    }
    out = w;
    return GL_OK;
}

// A finished request that asked for its factor: the workspace w becomes a
// registered factor the queue may evict (least recently used first) when its
// admission needs room.  Returns false (w stays with the queue, the result
// carries no factor) when the factor object cannot be made.
bool hand_over(lq_queue *q, Request *r, Work &w)
{
    gl_factor *f = factor_adopt(q->ctx, w, r->th, r->o, q);
    if (!f) return false;
    r->res.factor = f;
    w = Work{};
    return true;
}

// Frees memory for a request needing `need` more bytes: idle pooled and slot
// workspaces first (keep_slot's excepted), then factors handed out by this
// queue, least recently used first.  Returns whether held + need now fits.
bool make_room(lq_queue *q, size_t need, size_t mine, const Slot *keep_slot)
{
    for (Work *w : q->pool) {
        q->ctx->used -= w->bytes();
        w->release();
        delete w;
    }
    q->pool.clear();
    for (Slot &sl : q->slots)
        if (!sl.req && &sl != keep_slot && slot_bytes(sl)) {
            q->ctx->used -= slot_bytes(sl);
            sl.w.release();
        }
    size_t held = held_bytes(q);
    if (held - mine + need <= q->budget) return true;
    evict_factors(q->ctx, q, held - mine + need - q->budget);
    return held_bytes(q) - mine + need <= q->budget;
}

// Enqueue one tick of cohort c: every resident advances by one step.
int build_tick(lq_queue *q, Cohort &co)
{
    TickBuf &tb = co.ring[co.ring_next];
    if (tb.busy) return GL_EBUSY;
    const int count = (int)co.residents.size();
    for (int i = 0; i < count; ++i) {
        Resident &r = co.residents[i];
        Work &w = *r.w;
        BatchReq &d = tb.host[i];
        d.tiles = w.tiles;
        d.x = w.x;
        d.y = w.y;
        d.v = w.v;
        d.dinv = w.dinv_k(r.k);
        d.logsum = w.logsum;
        d.quad = w.quad;
        d.info = w.info;
        d.res = w.res;
        const int64_t n = r.req->ds->n;
        d.sx = r.req->ds->buf;
        d.sy = d.sx + n;
        d.sz = d.sy + n;
        d.th = r.req->th;
        d.geo = geom_of(r.req->o);
        d.n = w.n;
        d.nt = w.nt;
        d.npad = w.npad;
        d.k = r.k;
        d.is_new = r.is_new ? 1 : 0;
        d.finishing = (r.k == w.nt - 1) ? 1 : 0;
    }
    hipStream_t s = co.s;
    int launches = 0;
    const auto h0 = std::chrono::steady_clock::now();
    GL_HIP_TRY(hipEventRecord(tb.start, s));
    const int rc = enqueue_step(tb.host, tb.dev, count, TICK_B, s, &launches);
    if (rc != GL_OK) return rc;
    tb.finishing.clear();
    GL_HIP_TRY(hipGetLastError());
    std::vector<Resident> keep;
    keep.reserve(co.residents.size());
    for (int i = 0; i < count; ++i) {
        Resident r = co.residents[i];
        r.is_new = false;
        if (tb.host[i].finishing) {
            GL_HIP_TRY(hipMemcpyAsync(&tb.res_h[tb.finishing.size()], r.w->res, sizeof(DevResult),
                                      hipMemcpyDeviceToHost, s));
            tb.finishing.push_back(r);
        } else {
            r.k += 1;
            keep.push_back(r);
        }
    }
    co.residents.swap(keep);
    GL_HIP_TRY(hipEventRecord(tb.done, s));
    tb.busy = true;
    co.ticks.push_back(co.ring_next);
    co.ring_next = (co.ring_next + 1) % TICK_RING;
    q->fused += launches;
    q->ticks += 1;
    q->host_us += std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - h0).count();
    return GL_OK;
}

// Deliver the results of completed ticks of cohort c (oldest first).
void retire_ticks(lq_queue *q, Cohort &co)
{
    while (!co.ticks.empty()) {
        TickBuf &tb = co.ring[co.ticks.front()];
        hipError_t e = hipEventQuery(tb.done);
        if (e == hipErrorNotReady) return;
        float ms = 0.f;
        if (e == hipSuccess && hipEventElapsedTime(&ms, tb.start, tb.done) == hipSuccess) q->device_ms += ms;
        if (e == hipSuccess && co.last_done && hipEventElapsedTime(&ms, co.last_done, tb.start) == hipSuccess &&
            ms > 0.f)
            q->gap_ms += ms;
        co.last_done = tb.done;
        for (size_t i = 0; i < tb.finishing.size(); ++i) {
            Resident &r = tb.finishing[i];
            Request *req = r.req;
            const DevResult &d = tb.res_h[i];
            --q->inflight;
            ++q->completed;
            if (e != hipSuccess) {
                finish(q, req, GL_EHIP);
            } else {
                req->res.loglik = d.loglik;
                req->res.logdet = d.logdet;
                req->res.quad = d.quad;
                req->res.info = d.info;
                req->res.tile = TICK_B;
                req->res.factor = nullptr;
                if (!d.info && req->o.keep_factor && hand_over(q, req, *r.w)) {
                    delete r.w;  // its memory now belongs to the factor
                    r.w = nullptr;
                }
                finish(q, req, d.info ? GL_NOT_SPD : GL_OK);
            }
            if (r.w) q->pool.push_back(r.w);
        }
        tb.finishing.clear();
        tb.busy = false;
        co.ticks.pop_front();
    }
}


// A slot's stream, its lane (lookahead and forward-solve streams), event and
// pinned result are created on its first request.  The usual serving load (binary64, n <= small_n) runs
// through the fused launches on the two cohort streams only, so a queue adds
// two streams to the process, within the four hardware queues a process gets
// by default, and the cohorts do not share a hardware queue with idle slots.
static int slot_open(Slot &sl)
{
    if (sl.s) return GL_OK;
    GL_HIP_TRY(hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking));
    if (sl.ln.create() != GL_OK) return GL_EHIP;
    GL_HIP_TRY(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    GL_HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&sl.res_h), sizeof(DevResult), hipHostMallocDefault));
    return GL_OK;
}

// Launch request r on slot sl (queue lock released by the caller).
int launch_on_slot(gl_context *ctx, Slot &sl, Request *r)
{
    int rc0 = slot_open(sl);
    if (rc0 != GL_OK) return rc0;
    const int64_t n = r->ds->n;
    const int b = pick_tile(n, r->o.tile);
    int rc = sl.w.ensure(ctx, n, b, r->o.precision);
    if (rc != GL_OK) return rc;
    const double *x = r->ds->buf, *y = x + n, *z = y + n;
    stage_inputs(sl.w, x, y, z, r->o.reorder, sl.s);
    rc = eval_launch(sl.ln, sl.w, r->th, r->o, sl.s, sl.res_h);
    if (rc != GL_OK) return rc;
    GL_HIP_TRY(hipEventRecord(sl.done, sl.s));
    return GL_OK;
}

void scheduler(lq_queue *q)
{
    hipSetDevice(q->ctx->device);
    std::unique_lock<std::mutex> lk(q->mu);
    for (;;) {
        // retire finished slots
        for (Slot &sl : q->slots) {
            if (!sl.req) continue;
            hipError_t e = hipEventQuery(sl.done);
            if (e == hipErrorNotReady) continue;
            Request *r = sl.req;
            sl.req = nullptr;
            --q->inflight;
            ++q->completed;
            if (e != hipSuccess) {
                finish(q, r, GL_EHIP);
                continue;
            }
            r->res.loglik = sl.res_h->loglik;
            r->res.logdet = sl.res_h->logdet;
            r->res.quad = sl.res_h->quad;
            r->res.info = sl.res_h->info;
            r->res.tile = sl.w.b;
            r->res.factor = nullptr;
            if (!sl.res_h->info && r->o.keep_factor) hand_over(q, r, sl.w);
            finish(q, r, sl.res_h->info ? GL_NOT_SPD : GL_OK);
        }
        for (Cohort &c : q->co) retire_ticks(q, c);
        // admit queued requests in arrival order: batched residents or free slots
        while (!q->queue.empty()) {
            Request *head = q->queue.front();
            if (batch_eligible(q, head)) {
                Cohort *dst = &q->co[0];
                for (Cohort &c : q->co)
                    if (c.residents.size() < dst->residents.size()) dst = &c;
                if (q->inflight >= q->cfg.max_inflight || (int)dst->residents.size() >= TICK_MAX) break;
                const size_t need = work_bytes(head->ds->n, TICK_B, GL_FP64);
                bool have = false;
                for (Work *w : q->pool) have = have || w->bytes() >= need;
                if (!have && held_bytes(q) + need > q->budget && !make_room(q, need, 0, nullptr)) {
                    if (q->inflight > 0) break;  // wait for running requests to free memory
                    q->queue.pop_front();
                    finish(q, head, GL_ENOMEM);  // larger than the whole budget
                    continue;
                }
                Work *w = nullptr;
                int rc = take_work(q, head->ds->n, w);
                q->queue.pop_front();
                if (rc != GL_OK) {
                    finish(q, head, rc);
                    continue;
                }
                head->state = RUNNING;
                Resident res;
                res.req = head;
                res.w = w;
                dst->residents.push_back(res);
                ++q->inflight;
                if (q->inflight > q->peak_inflight) q->peak_inflight = q->inflight;
                continue;
            }
            if (q->inflight >= q->cfg.max_inflight) break;
            Slot *free_slot = nullptr;
            for (Slot &sl : q->slots)
                if (!sl.req) {
                    free_slot = &sl;
                    break;
                }
            if (!free_slot) break;
            Request *r = q->queue.front();
            const int64_t n = r->ds->n;
            const size_t need = work_bytes(n, pick_tile(n, r->o.tile), r->o.precision);
            size_t held = held_bytes(q);
            const size_t mine = slot_bytes(*free_slot);
            if (need > mine && held - mine + need > q->budget && !make_room(q, need, mine, free_slot)) {
                if (q->inflight > 0) break;  // wait for running requests to free memory
                q->queue.pop_front();
                finish(q, r, GL_ENOMEM);  // larger than the whole budget
                continue;
            }
            q->queue.pop_front();
            r->state = RUNNING;
            free_slot->req = r;
            ++q->inflight;
            if (q->inflight > q->peak_inflight) q->peak_inflight = q->inflight;
            lk.unlock();
            int rc = launch_on_slot(q->ctx, *free_slot, r);
            lk.lock();
            if (rc != GL_OK) {
                free_slot->req = nullptr;
                --q->inflight;
                finish(q, r, rc);
            }
            const size_t h = held_bytes(q);
            if (h > q->peak_bytes) q->peak_bytes = h;
        }
        bool ticked = false;
        for (Cohort &c : q->co) {
            if (c.residents.empty() || (int)c.ticks.size() >= TICK_DEPTH) continue;
            const int rc = build_tick(q, c);
            if (rc != GL_OK && rc != GL_EBUSY) {
                for (Resident &r : c.residents) {
                    --q->inflight;
                    finish(q, r.req, rc);
                    q->pool.push_back(r.w);
                }
                c.residents.clear();
            }
            ticked = ticked || rc == GL_OK;
        }
        if (ticked) {
            const size_t h = held_bytes(q);
            if (h > q->peak_bytes) q->peak_bytes = h;
            continue;
        }
        if (q->stop && q->queue.empty() && q->inflight == 0) break;
        if (q->inflight > 0) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            q->cv_work.wait(lk, [q] { return q->stop || !q->queue.empty(); });
        }
    }
}

}  // namespace

extern "C" {

int gl_dataset_register(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n,
                        uint64_t *ds_h)
{
    if (!ctx || !x || !y || !z || n < 1 || !ds_h) return GL_EINVAL;
    GL_HIP_TRY(hipSetDevice(ctx->device));
    ServeState *st = serve_state(ctx);
    const size_t bytes = 3 * (size_t)n * sizeof(double);
    if (ctx->used.load() + bytes > ctx->budget) return GL_ENOMEM;
    Dataset *d = new Dataset();
    d->n = n;
    if (hipMalloc(reinterpret_cast<void **>(&d->buf), bytes) != hipSuccess) {
        delete d;
        return GL_ENOMEM;
    }
    ctx->used += bytes;
    hipError_t e = hipMemcpy(d->buf, x, n * sizeof(double), hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(d->buf + n, y, n * sizeof(double), hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(d->buf + 2 * n, z, n * sizeof(double), hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
        hipFree(d->buf);
        ctx->used -= bytes;
        delete d;
        return gl_hip_fail(e, "gl_dataset_register copy");
    }
    std::lock_guard<std::mutex> lk(st->mu);
    d->id = st->next++;
    st->sets[d->id] = d;
    *ds_h = d->id;
    return GL_OK;
}

int gl_dataset_release(gl_context *ctx, uint64_t id)
{
    if (!ctx) return GL_EINVAL;
    ServeState *st = serve_state(ctx);
    Dataset *d = nullptr;
    std::vector<lq_queue *> queues;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        auto it = st->sets.find(id);
        if (it == st->sets.end()) return GL_EINVAL;
        d = it->second;
        st->sets.erase(it);
        st->graveyard.push_back(d);
        queues = st->queues;
    }
    for (lq_queue *q : queues) {
        std::lock_guard<std::mutex> lk(q->mu);
        for (auto it = q->queue.begin(); it != q->queue.end();) {
            if ((*it)->ds == d) {
                Request *r = *it;
                it = q->queue.erase(it);
                finish(q, r, GL_ECANCELED);
            } else {
                ++it;
            }
        }
    }
    d->dropped = true;
    if (d->refs.load() == 0) {
        hipSetDevice(ctx->device);
        d->free_once();
    }
    ctx->used -= 3 * (size_t)d->n * sizeof(double);
    return GL_OK;
}

void lq_config_default(lq_config *c)
{
    if (!c) return;
    c->max_inflight = 32;
    c->streams = 4;
    c->batch_small = 1;
    c->small_n = 16384;
    c->hbm_budget_bytes = 0;
}

int lq_create(gl_context *ctx, const lq_config *cfg, lq_queue **out)
{
    if (!ctx || !out) return GL_EINVAL;
    lq_config c;
    lq_config_default(&c);
    if (cfg) c = *cfg;
    if (c.max_inflight < 1 || c.max_inflight > 64 || c.streams < 1 || c.streams > 8) return GL_EINVAL;
    GL_HIP_TRY(hipSetDevice(ctx->device));
    lq_queue *q = new lq_queue();
    q->ctx = ctx;
    q->cfg = c;
    q->budget = c.hbm_budget_bytes ? c.hbm_budget_bytes : ctx->budget;
    q->slots.resize(c.streams);  // their streams are created on first use (slot_open)
    for (Cohort &c : q->co) {
        bool ok = hipStreamCreateWithFlags(&c.s, hipStreamNonBlocking) == hipSuccess;
        for (TickBuf &tb : c.ring)
            ok = ok &&
                 hipHostMalloc(reinterpret_cast<void **>(&tb.host), TICK_MAX * sizeof(BatchReq),
                               hipHostMallocDefault) == hipSuccess &&
                 hipMalloc(reinterpret_cast<void **>(&tb.dev), TICK_MAX * sizeof(BatchReq)) == hipSuccess &&
                 hipHostMalloc(reinterpret_cast<void **>(&tb.res_h), TICK_MAX * sizeof(DevResult),
                               hipHostMallocDefault) == hipSuccess &&
                 hipEventCreate(&tb.start) == hipSuccess && hipEventCreate(&tb.done) == hipSuccess;
        if (!ok) {
            q->stop = true;
            lq_destroy(q);
            return GL_EHIP;
        }
    }
    ServeState *st = serve_state(ctx);
    {
        std::lock_guard<std::mutex> lk(st->mu);
        st->queues.push_back(q);
    }
    q->thr = std::thread(scheduler, q);
    *out = q;
    return GL_OK;
}

int lq_submit(lq_queue *q, uint64_t ds, gl_theta th, const gl_opts *opts, uint64_t *ticket)
{
    if (!q || !ticket || !valid_theta(th)) return GL_EINVAL;
    gl_opts o;
    gl_opts_default(&o);
    if (opts) o = *opts;
    o.graph = 0;  // the queue schedules its own launches
    if (!valid_opts(o) || !valid_theta_for(th, o) || o.ind_tiles != 0) return GL_EINVAL;
    o = resolved_opts(o);
    ServeState *st = serve_state(q->ctx);
    Request *r = new Request();
    {
        std::lock_guard<std::mutex> lk(st->mu);
        auto it = st->sets.find(ds);
        if (it == st->sets.end()) {
            delete r;
            return GL_EINVAL;
        }
        r->ds = it->second;
        r->ds->refs += 1;
    }
    r->th = th;
    r->o = o;
    {
        std::lock_guard<std::mutex> lk(q->mu);
        if (q->stop) {
            r->ds->refs -= 1;
            delete r;
            return GL_ECANCELED;
        }
        r->ticket = q->next_ticket++;
        q->reqs[r->ticket] = r;
        q->queue.push_back(r);
        *ticket = r->ticket;
    }
    q->cv_work.notify_one();
    return GL_OK;
}

static int take_result(lq_queue *q, std::unordered_map<uint64_t, Request *>::iterator it, gl_result *res)
{
    Request *r = it->second;
    if (res) *res = r->res;
    const int st = r->res.status;
    q->reqs.erase(it);
    delete r;
    return st;
}

int lq_poll(lq_queue *q, uint64_t ticket, gl_result *res)
{
    if (!q) return GL_EINVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    auto it = q->reqs.find(ticket);
    if (it == q->reqs.end()) return GL_EINVAL;
    if (it->second->state != DONE) return GL_EBUSY;
    return take_result(q, it, res);
}

int lq_wait(lq_queue *q, uint64_t ticket, gl_result *res, int64_t timeout_us)
{
    if (!q) return GL_EINVAL;
    std::unique_lock<std::mutex> lk(q->mu);
    auto it = q->reqs.find(ticket);
    if (it == q->reqs.end()) return GL_EINVAL;
    Request *r = it->second;
    auto ready = [r] { return r->state == DONE; };
    if (timeout_us < 0) {
        q->cv_done.wait(lk, ready);
    } else if (!q->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return GL_ETIMEDOUT;
    }
    return take_result(q, q->reqs.find(ticket), res);
}

int lq_cancel(lq_queue *q, uint64_t ticket)
{
    if (!q) return GL_EINVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    auto it = q->reqs.find(ticket);
    if (it == q->reqs.end()) return GL_EINVAL;
    Request *r = it->second;
    if (r->state != QUEUED) return GL_EBUSY;
    for (auto qi = q->queue.begin(); qi != q->queue.end(); ++qi)
        if (*qi == r) {
            q->queue.erase(qi);
            break;
        }
    finish(q, r, GL_ECANCELED);
    return GL_OK;
}

int lq_stats(lq_queue *q, uint64_t *completed, size_t *peak_bytes, int32_t *peak_inflight,
             uint64_t *fused_launches)
{
    if (!q) return GL_EINVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    if (completed) *completed = q->completed;
    if (peak_bytes) *peak_bytes = q->peak_bytes;
    if (peak_inflight) *peak_inflight = q->peak_inflight;
    if (fused_launches) *fused_launches = q->fused;
    return GL_OK;
}

int lq_tick_stats(lq_queue *q, uint64_t *ticks, double *host_us, double *device_ms, double *gap_ms)
{
    if (!q) return GL_EINVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    if (ticks) *ticks = q->ticks;
    if (host_us) *host_us = q->host_us;
    if (device_ms) *device_ms = q->device_ms;
    if (gap_ms) *gap_ms = q->gap_ms;
    return GL_OK;
}

int lq_destroy(lq_queue *q)
{
    if (!q) return GL_EINVAL;
    {
        std::lock_guard<std::mutex> lk(q->mu);
        q->stop = true;
        while (!q->queue.empty()) {
            Request *r = q->queue.front();
            q->queue.pop_front();
            finish(q, r, GL_ECANCELED);
        }
    }
    q->cv_work.notify_all();
    if (q->thr.joinable()) q->thr.join();
    if (q->ctx->serve) {
        std::lock_guard<std::mutex> lk(q->ctx->serve->mu);
        auto &v = q->ctx->serve->queues;
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i] == q) {
                v.erase(v.begin() + i);
                break;
            }
    }
    hipSetDevice(q->ctx->device);
    for (Cohort &c : q->co)
        if (c.s) hipStreamSynchronize(c.s);
    for (Work *w : q->pool) {
        q->ctx->used -= w->bytes();
        w->release();
        delete w;
    }
    q->pool.clear();
    for (Cohort &c : q->co) {
        for (TickBuf &tb : c.ring) {
            if (tb.host) hipHostFree(tb.host);
            if (tb.dev) hipFree(tb.dev);
            if (tb.res_h) hipHostFree(tb.res_h);
            if (tb.start) hipEventDestroy(tb.start);
            if (tb.done) hipEventDestroy(tb.done);
        }
        if (c.s) hipStreamDestroy(c.s);
    }
    for (Slot &sl : q->slots) {
        if (sl.s) hipStreamSynchronize(sl.s);
        q->ctx->used -= slot_bytes(sl);
        sl.w.release();
        sl.ln.destroy();
        if (sl.s) hipStreamDestroy(sl.s);
        if (sl.done) hipEventDestroy(sl.done);
        if (sl.res_h) hipHostFree(sl.res_h);
    }
    for (auto &kv : q->reqs) delete kv.second;
    detach_factors(q->ctx, q);  // factors already handed out stay with their owners
    delete q;
    return GL_OK;
}

}  // extern "C"
