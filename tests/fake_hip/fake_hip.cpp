// Host implementation of the HIP stand-in declared in hip/hip_runtime.h (see
// there).  Test infrastructure only.
#include <hip/hip_runtime.h>

#include <random>

namespace {
thread_local std::mt19937 rng(12345);
std::atomic<int> next_stream{1};
}  // namespace

hipError_t hipGetDeviceCount(int *n)
{
    *n = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int)
{
    memset(p, 0, sizeof(*p));
    strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
    p->multiProcessorCount = 256;
    return hipSuccess;
}
hipError_t hipMemGetInfo(size_t *freeb, size_t *total)
{
    *freeb = (size_t)8 << 30;
    *total = (size_t)8 << 30;
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t n)
{
    *p = n ? aligned_alloc(256, (n + 255) / 256 * 256) : nullptr;
    return (*p || !n) ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p)
{
    free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void *p) { return hipFree(p); }
hipError_t hipMallocAsync(void **p, size_t n, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipFreeAsync(void *p, hipStream_t) { return hipFree(p); }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind)
{
    if (n) memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t)
{
    return hipMemcpy(d, s, n, k);
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    *s = new FakeStream{next_stream++};
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = new FakeEvent();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t)
{
    e->pending.store((int)(rng() % 3));
    e->seq.fetch_add(1);
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e)
{
    int p = e->pending.load();
    while (p > 0) {
        if (e->pending.compare_exchange_weak(p, p - 1)) return hipErrorNotReady;
    }
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    e->pending.store(0);
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t)
{
    *ms = 0.01f;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "fake HIP error"; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorInvalidValue; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g)
{
    *g = nullptr;
    return hipErrorInvalidValue;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t, void *, char *, size_t)
{
    *e = nullptr;
    return hipErrorInvalidValue;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
