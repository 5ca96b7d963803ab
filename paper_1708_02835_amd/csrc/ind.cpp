// Independent-blocks (IND) approximation, Sec. 6.8: the tiles outside the
// diagonal super tiles of s×s tiles are annihilated, so Σ is block diagonal
// with blocks of s·b consecutive locations and l(θ) is the sum of the exact
// log-likelihoods of the blocks.  Nothing outside the blocks is generated or
// factored: the blocks are independent factorisations of s tile columns each
// (the last one possibly shorter), advanced together through the fused
// multi-factorisation launches, one tile step per launch group.
//
// Kriging under the same approximation (the exact-versus-IND prediction
// comparison of the paper's experiments, with Eq. (5)): applied to the
// covariance of all locations, observed and held-out alike, the blocks are
// independent fields, so each held-out value is predicted from the observed
// values of its own block, Z_M = Σ_MO Σ_OO⁻¹ Z_O, through the block's factor
// (backward substitution of w = L⁻¹ Z_O).
#include <algorithm>
#include <vector>

#include "batch.hpp"
#include "engine.hpp"

namespace gl {

// Sums the per-block results in block order; info of the first failing block,
// as a global 1-based column.
__global__ void ind_total_kernel(const DevResult *__restrict__ r, int64_t nblk, int64_t block,
                                 DevResult *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double l = 0.0, ld = 0.0, q = 0.0;
    int64_t info = 0;
    for (int64_t i = 0; i < nblk; ++i) {
        if (info == 0 && r[i].info != 0) info = i * block + r[i].info;
        l += r[i].loglik;
        ld += r[i].logdet;
        q += r[i].quad;
    }
    out->info = info;
    out->loglik = info ? -INFINITY : l;
    out->logdet = info ? NAN : ld;
    out->quad = info ? NAN : q;
}

// The blocks of one IND factorisation: one descriptor per block (factor
// tiles, padded coordinates, w = L⁻¹ Z of the block in v), the locations the
// blocks were cut from (input or Morton order) and the device total.
struct IndPlan {
    int b = 0;
    int64_t nblk = 0;
    std::vector<BatchReq> proto;
    std::vector<int64_t> start, nb, ntb;
    const double *sx = nullptr, *sy = nullptr;
    DevResult *total = nullptr;
};

// Enqueues the factorisation of the blocks [start[i], start[i] + count[i])
// of the locations (each count >= 1, at most bt tiles of b) and the
// fixed-order sum of the per-block results into p.total (all on s).  With
// reorder the locations are first put in Morton order.
static int ind_factor(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n, gl_theta th,
                      const gl_opts &o, int b, int64_t bt, const std::vector<int64_t> &start,
                      const std::vector<int64_t> &count, bool reorder, hipStream_t s, IndPlan &p)
{
    const int64_t nblk = (int64_t)start.size();
    const int64_t block = bt * b;  // uniform block length (the likelihood's), for the reported column
    // layout (in doubles): descriptors | totals | per-block results, info |
    // per block: tiles, x, y, v, logsum, quad, dinv | reordered inputs, keys
    const size_t desc_d = ((size_t)nblk * sizeof(BatchReq) + 15) / 16 * 2;
    size_t off = desc_d + 8 + 8 * (size_t)nblk + 8 * (size_t)nblk;
    std::vector<size_t> boff(nblk);
    std::vector<int64_t> nb(nblk), ntb(nblk);
    for (int64_t i = 0; i < nblk; ++i) {
        nb[i] = count[i];
        ntb[i] = ceil_div(nb[i], b);
        const int64_t npb = ntb[i] * b;
        boff[i] = off;
        off += (size_t)tile_count(ntb[i]) * b * b + 3 * npb + 2 * ntb[i] + (ntb[i] & 1) + 64 * npb;
    }
    const size_t morton_off = off;
    if (reorder) off += 3 * (size_t)n + (n & 1) + (size_t)npow2_of(n) + 4;
    const size_t bytes = off * sizeof(double);
    if (bytes > ctx->ind_cap) {
        const size_t old = ctx->ind_cap;
        if (ctx->used.load() - old + bytes > ctx->budget) return GL_ENOMEM;
        if (ctx->ind_buf) hipFree(ctx->ind_buf);
        ctx->ind_buf = nullptr;
        ctx->ind_cap = 0;
        ctx->used -= old;
        if (hipMalloc(&ctx->ind_buf, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return GL_ENOMEM;
        }
        ctx->ind_cap = bytes;
        ctx->used += bytes;
    }
    double *base = static_cast<double *>(ctx->ind_buf);
    BatchReq *ddesc = reinterpret_cast<BatchReq *>(base);
    DevResult *total = reinterpret_cast<DevResult *>(base + desc_d);
    DevResult *bres = reinterpret_cast<DevResult *>(base + desc_d + 8);
    int64_t *binfo = reinterpret_cast<int64_t *>(base + desc_d + 8 + 8 * nblk);
    const double *sx = x, *sy = y, *sz = z;
    if (reorder) {
        double *xo = base + morton_off, *yo = xo + n, *zo = yo + n;
        uint64_t *keys = reinterpret_cast<uint64_t *>(zo + n + (n & 1));
        launch_morton_order(x, y, z, n, n, keys, xo, yo, zo, nullptr, s);  // unpadded output
        sx = xo;
        sy = yo;
        sz = zo;
    }
    std::vector<BatchReq> proto(nblk);
    for (int64_t i = 0; i < nblk; ++i) {
        BatchReq &d = proto[i];
        const int64_t npb = ntb[i] * b;
        double *p = base + boff[i];
        d.tiles = p;
        p += (size_t)tile_count(ntb[i]) * b * b;
        d.x = p;
        d.y = p + npb;
        d.v = p + 2 * npb;
        p += 3 * npb;
        d.logsum = p;
        d.quad = p + ntb[i];
        p += 2 * ntb[i] + (ntb[i] & 1);
        d.dinv = p;
        d.info = binfo + 8 * i;
        d.res = bres + i;
        d.sx = sx + start[i];
        d.sy = sy + start[i];
        d.sz = sz + start[i];
        d.th = th;
        d.geo = geom_of(o);
        d.n = nb[i];
        d.nt = ntb[i];
        d.npad = npb;
    }
    // The descriptors of every step go to pinned host memory owned by the
    // context (one region per step), which the asynchronous copies read until
    // the stream passes them; the previous call's copies are waited for
    // before the memory is rewritten or replaced.
    const size_t entries = (size_t)bt * (size_t)nblk;
    if (ctx->ind_done) GL_HIP_TRY(hipEventSynchronize(ctx->ind_done));
    else GL_HIP_TRY(hipEventCreateWithFlags(&ctx->ind_done, hipEventDisableTiming));
    if (entries > ctx->ind_host_cap) {
        if (ctx->ind_host) GL_HIP_TRY(hipHostFree(ctx->ind_host));
        ctx->ind_host = nullptr;
        ctx->ind_host_cap = 0;
        GL_HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&ctx->ind_host), entries * sizeof(BatchReq),
                                 hipHostMallocDefault));
        ctx->ind_host_cap = entries;
    }
    BatchReq *h = ctx->ind_host;
    for (int64_t k = 0; k < bt; ++k) {
        int cnt = 0;
        for (int64_t i = 0; i < nblk; ++i) {
            if (k >= ntb[i]) continue;  // the last block may have fewer tile columns
            BatchReq &d = h[cnt++];
            d = proto[i];
            d.dinv = proto[i].dinv + k * 64 * (int64_t)b;
            d.k = k;
            d.is_new = k == 0;
            d.finishing = k == ntb[i] - 1;
        }
        if (cnt == 0) break;
        const int rc = enqueue_step(h, ddesc, cnt, b, s, nullptr);
        if (rc != GL_OK) return rc;
        h += cnt;
    }
    GL_HIP_TRY(hipEventRecord(ctx->ind_done, s));
    ind_total_kernel<<<1, 64, 0, s>>>(bres, nblk, block, total);
    GL_HIP_TRY(hipGetLastError());
    p.b = b;
    p.nblk = nblk;
    p.proto = std::move(proto);
    p.start = start;
    p.nb = std::move(nb);
    p.ntb = std::move(ntb);
    p.sx = sx;
    p.sy = sy;
    p.total = total;
    return GL_OK;
}

int ind_eval(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n, gl_theta th,
             const gl_opts &o, gl_result *res, hipStream_t s)
{
    const int b = pick_tile(n, o.tile);
    const int64_t block = o.ind_tiles * (int64_t)b;
    std::vector<int64_t> start, count;
    for (int64_t a = 0; a < n; a += block) {
        start.push_back(a);
        count.push_back(std::min(block, n - a));
    }
    IndPlan p;
    const int rc = ind_factor(ctx, x, y, z, n, th, o, b, o.ind_tiles, start, count, o.reorder != 0, s, p);
    if (rc != GL_OK) return res->status = rc;
    GL_HIP_TRY(hipMemcpyAsync(ctx->res_h, p.total, sizeof(DevResult), hipMemcpyDeviceToHost, s));
    GL_HIP_TRY(hipStreamSynchronize(s));
    fill_result(res, *ctx->res_h, p.b);
    return res->status;
}

int ind_krige(gl_context *ctx, const double *x, const double *y, const double *z, const int64_t *kcount,
              const double *xnew, const double *ynew, const int64_t *mcount, int64_t nblocks, gl_theta th,
              const gl_opts &o, int b, double *znew, hipStream_t s)
{
    // blocks that observe something are factored; the others predict 0
    std::vector<int64_t> start, count, kstart(nblocks + 1, 0), mstart(nblocks + 1, 0), slot(nblocks, -1);
    for (int64_t B = 0; B < nblocks; ++B) {
        kstart[B + 1] = kstart[B] + kcount[B];
        mstart[B + 1] = mstart[B] + mcount[B];
        if (kcount[B] > 0) {
            slot[B] = (int64_t)start.size();
            start.push_back(kstart[B]);
            count.push_back(kcount[B]);
        }
    }
    const int64_t n = kstart[nblocks];
    IndPlan p;
    if (!start.empty()) {
        int rc = ind_factor(ctx, x, y, z, n, th, o, b, o.ind_tiles, start, count, false, s, p);
        if (rc != GL_OK) return rc;
        GL_HIP_TRY(hipMemcpyAsync(ctx->res_h, p.total, sizeof(DevResult), hipMemcpyDeviceToHost, s));
        GL_HIP_TRY(hipStreamSynchronize(s));
        if (ctx->res_h->info != 0) return GL_NOT_SPD;
        // X = L⁻ᵀ w within each block, in place
        for (int64_t i = 0; i < p.nblk; ++i) {
            const BatchReq &d = p.proto[i];
            for (int64_t k = p.ntb[i] - 1; k >= 0; --k) {
                launch_bwd_diag(d.tiles, p.b, k, d.v, s);
                launch_bwd_update(d.tiles, p.b, k, d.v, s);
            }
        }
    }
    // each block's held-out values from its own observed values
    int64_t part_len = 1;
    for (int64_t B = 0; B < nblocks; ++B)
        if (mcount[B] > 0 && kcount[B] > 0) part_len = std::max(part_len, mcount[B] * krige_chunks(kcount[B]));
    double *part = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&part), (size_t)part_len * sizeof(double), s) != hipSuccess) {
        (void)hipGetLastError();
        return GL_ENOMEM;
    }
    for (int64_t B = 0; B < nblocks; ++B) {
        if (mcount[B] == 0) continue;
        double *out = znew + mstart[B];
        if (kcount[B] == 0) {
            launch_fill(out, mcount[B], 0.0, s);
            continue;
        }
        const int64_t nchunk = krige_chunks(kcount[B]);
        launch_krige(x + kstart[B], y + kstart[B], kcount[B], p.proto[slot[B]].v, th, geom_of(o), xnew + mstart[B],
                     ynew + mstart[B], mcount[B], part, nchunk, s);
        launch_krige_reduce(part, mcount[B], nchunk, out, s);
    }
    GL_HIP_TRY(hipGetLastError());
    GL_HIP_TRY(hipFreeAsync(part, s));
    return GL_OK;
}

}  // namespace gl
