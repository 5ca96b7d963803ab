// Likelihood evaluation without device allocation, for callers that cannot
// allocate (code under stream capture, tight serving loops, hosts that forbid
// hipMalloc).  It runs the same kernels as loglik_eval in binary64 (Alg. 2),
// with the workspace (packed lower tiles and vectors) placed in a file-scope
// device array instead of memory the context allocates.
//
// The array is part of this file's code object: each device the library runs
// on holds its own copy, at its own address, until the process ends.  Host
// code never passes the array's name to a kernel (on the host that name is a
// stand-in, not a device address); it passes the address hipGetSymbolAddress
// returned for the device, looked up once per device when a context is
// created there.  Every call on a device shares that device's array, so calls
// that overlap on one device (from any context) race.

#include <mutex>
#include <string.h>

#include "engine.hpp"

static __device__ __align__(256) double scratch[GL_SCRATCH_BYTES / sizeof(double)];

namespace gl {

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of this device's scratch array; the device must be current.
int scratch_init(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return GL_ENODEV;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[device]) {
        void *p = nullptr;
        GL_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        scratch_dev[device] = p;
    }
    *out = scratch_dev[device];
    return GL_OK;
}

}  // namespace gl

using namespace gl;

extern "C" int loglik_eval_noalloc(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n,
                                   gl_theta th, const gl_opts *opts, gl_result *res, void *stream)
{
    if (!res) return GL_EINVAL;
    memset(res, 0, sizeof(*res));
    gl_opts o;
    gl_opts_default(&o);
    if (opts) o = *opts;
    if (!ctx || !x || !y || !z || n < 1 || !valid_opts(o) || !valid_theta(th) || o.precision != GL_FP64 ||
        o.keep_factor || o.ind_tiles || o.graph) {
        res->status = GL_EINVAL;
        return GL_EINVAL;
    }
    o = resolved_opts(o);
    const int b = pick_tile(n, o.tile);
    Work w;
    if (w.bind(ctx->scratch, ctx->scratch ? GL_SCRATCH_BYTES : 0, n, b) != GL_OK) {
        res->status = ctx->scratch ? GL_E2BIG : GL_EHIP;
        return res->status;
    }
    GL_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Lanes ln = ctx->lanes;
    ln.prof = nullptr;  // kernel timing creates events; this path creates nothing
    stage_inputs(w, x, y, z, o.reorder, s);
    int rc = eval_launch(ln, w, th, o, s, ctx->res_h, nullptr);
    if (rc == GL_OK && hipStreamSynchronize(s) != hipSuccess) rc = GL_EHIP;
    if (rc != GL_OK) {
        res->status = rc;
        return rc;
    }
    fill_result(res, *ctx->res_h, b);
    return res->status;
}
