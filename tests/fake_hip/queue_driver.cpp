// Concurrency check of the request queue on the CPU (built against the HIP
// stand-in of this folder, run under ThreadSanitizer and AddressSanitizer by
// tests/test_queue_fake.py).  Test infrastructure only.
//
// Client threads submit likelihood requests on several datasets with random
// θ, options (fused path, slots via mixed precision or another tile, kept
// factors) and ways of collecting the result (blocking wait, polling,
// cancellation); a further thread registers and drops a dataset while
// requests on it are queued.  The queue's budget holds only a few
// workspaces, so admission waits and releases kept factors.  Every delivered
// result is checked against the closed form the stand-in kernels compute
// (Σ = θ1·I), failing θ must report NOT_SPD, kriging on a kept factor must
// succeed or report GL_EVICTED.  Prints "ok" and exits 0 when every check
// passes.
#include <math.h>
#include <stdio.h>

#include <atomic>
#include <random>
#include <thread>
#include <vector>

#include "geolik.h"

namespace {

std::atomic<int> failures{0};
std::atomic<long> delivered{0}, cancelled{0}, evicted{0}, kriged{0};

#define CHECK(cond, ...)                      \
    do {                                      \
        if (!(cond)) {                        \
            fprintf(stderr, __VA_ARGS__);     \
            fputc('\n', stderr);              \
            failures++;                       \
        }                                     \
    } while (0)

struct Data {
    int64_t n;
    std::vector<double> x, y, z;
    uint64_t id = 0;
    double zz = 0.0;
};

double expected(const Data &d, gl_theta th)
{
    return -0.5 * d.zz / th.theta1 - 0.5 * (double)d.n * log(th.theta1) - 0.5 * (double)d.n * log(2.0 * M_PI);
}

Data make(int64_t n, unsigned seed)
{
    std::mt19937_64 r(seed);
    std::normal_distribution<double> nd;
    Data d;
    d.n = n;
    d.x.resize(n);
    d.y.resize(n);
    d.z.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        d.x[i] = (double)i;
        d.y[i] = 0.0;
        d.z[i] = nd(r);
        d.zz += d.z[i] * d.z[i];
    }
    return d;
}

void check_result(const Data &d, gl_theta th, int st, const gl_result &res)
{
    if (th.theta1 > 1000.0) {
        CHECK(st == GL_NOT_SPD && res.info >= 1 && res.factor == nullptr, "failing θ gave status %d info %ld", st,
              (long)res.info);
        return;
    }
    CHECK(st == GL_OK, "status %d for n=%ld", st, (long)d.n);
    if (st != GL_OK) return;
    const double e = expected(d, th);
    CHECK(fabs(res.loglik - e) <= 1e-10 * fabs(e), "l %.17g expected %.17g (n=%ld)", res.loglik, e, (long)d.n);
    delivered++;
}

}  // namespace

int main()
{
    gl_context *ctx = nullptr;
    if (gl_context_create(0, 0, &ctx) != GL_OK) {
        fprintf(stderr, "context\n");
        return 2;
    }
    std::vector<Data> sets;
    const int64_t sizes[] = {1, 200, 255, 700, 1300, 2100};
    for (int i = 0; i < 6; ++i) sets.push_back(make(sizes[i], 100 + i));
    for (Data &d : sets)
        CHECK(gl_dataset_register(ctx, d.x.data(), d.y.data(), d.z.data(), d.n, &d.id) == GL_OK, "register");
    lq_config cfg;
    lq_config_default(&cfg);
    cfg.max_inflight = 6;
    cfg.streams = 2;
    cfg.hbm_budget_bytes = 4 * gl_footprint_bytes(2100, 256, GL_FP64);
    lq_queue *q = nullptr;
    if (lq_create(ctx, &cfg, &q) != GL_OK) {
        fprintf(stderr, "queue\n");
        return 2;
    }

    const int threads = 6, per = 60;
    std::vector<std::thread> ts;
    for (int t = 0; t < threads; ++t)
        ts.emplace_back([&, t] {
            std::mt19937 r(1000 + t);
            std::uniform_real_distribution<double> u(0.0, 1.0);
            std::vector<gl_factor *> held;
            for (int k = 0; k < per; ++k) {
                const Data &d = sets[r() % sets.size()];
                gl_theta th{0.5 + 1.5 * u(r), 0.1, 0.5};
                if (u(r) < 0.05) th.theta1 = 5000.0;
                gl_opts o;
                gl_opts_default(&o);
                const double c = u(r);
                if (c < 0.15) o.precision = GL_MIXED_FP32;
                else if (c < 0.25) o.tile = 128;
                o.keep_factor = u(r) < 0.3;
                uint64_t tk = 0;
                const int sst = lq_submit(q, d.id, th, &o, &tk);
                CHECK(sst == GL_OK, "submit %d", sst);
                if (sst != GL_OK) continue;
                gl_result res;
                int st;
                const double how = u(r);
                if (how < 0.1) {
                    st = lq_cancel(q, tk);
                    CHECK(st == GL_OK || st == GL_EBUSY, "cancel %d", st);
                    st = lq_wait(q, tk, &res, -1);
                    if (st == GL_ECANCELED) {
                        cancelled++;
                        continue;
                    }
                } else if (how < 0.4) {
                    while ((st = lq_poll(q, tk, &res)) == GL_EBUSY) std::this_thread::yield();
                } else {
                    while ((st = lq_wait(q, tk, &res, 200)) == GL_ETIMEDOUT) {
                    }
                }
                check_result(d, th, st, res);
                if (res.factor) {
                    // krige on every factor this client holds (older ones may
                    // have been evicted), then keep at most three
                    held.push_back(res.factor);
                    for (gl_factor *f : held) {
                        double xn[3] = {0.5, 1.5, 2.5}, yn[3] = {0, 0, 0}, zn[3];
                        const int kst = krige_predict(ctx, f, xn, yn, 3, zn, nullptr, nullptr);
                        CHECK(kst == GL_OK || kst == GL_EVICTED, "krige %d", kst);
                        if (kst == GL_EVICTED) evicted++;
                        else kriged++;
                    }
                    if (held.size() > 3) {
                        CHECK(gl_factor_release(ctx, held.front()) == GL_OK, "release");
                        held.erase(held.begin());
                    }
                }
            }
            // half of the clients leave their factors to the context's destruction
            if (t % 2 == 0)
                for (gl_factor *f : held) CHECK(gl_factor_release(ctx, f) == GL_OK, "release");
        });
    // a dataset dropped while requests on it are queued: they are cancelled or served
    ts.emplace_back([&] {
        for (int k = 0; k < 20; ++k) {
            Data d = make(900, 500 + k);
            if (gl_dataset_register(ctx, d.x.data(), d.y.data(), d.z.data(), d.n, &d.id) != GL_OK) {
                failures++;
                continue;
            }
            std::vector<uint64_t> tk(4);
            for (uint64_t &t : tk) CHECK(lq_submit(q, d.id, gl_theta{1.0, 0.1, 0.5}, nullptr, &t) == GL_OK, "submit");
            CHECK(gl_dataset_release(ctx, d.id) == GL_OK, "dataset release");
            for (uint64_t t : tk) {
                gl_result res;
                const int st = lq_wait(q, t, &res, -1);
                if (st == GL_ECANCELED) cancelled++;
                else check_result(d, gl_theta{1.0, 0.1, 0.5}, st, res);
            }
        }
    });
    for (std::thread &t : ts) t.join();
    uint64_t completed = 0;
    CHECK(lq_stats(q, &completed, nullptr, nullptr, nullptr) == GL_OK, "stats");
    CHECK(lq_destroy(q) == GL_OK, "destroy");
    for (Data &d : sets) CHECK(gl_dataset_release(ctx, d.id) == GL_OK, "dataset release");
    gl_context_destroy(ctx);
    printf("delivered %ld cancelled %ld kriged %ld evicted %ld completed %lu failures %d\n", delivered.load(),
           cancelled.load(), kriged.load(), evicted.load(), (unsigned long)completed, failures.load());
    if (failures.load()) return 1;
    printf("ok\n");
    return 0;
}
