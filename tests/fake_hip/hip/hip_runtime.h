// A host-only stand-in for the HIP runtime, for building the library's host
// code (the request-queue scheduler, the context and factor bookkeeping) on
// the CPU under ThreadSanitizer and AddressSanitizer.  Test infrastructure
// only: device memory is host memory, streams execute every command at once
// (in call order), and an event reports "not ready" for a few queries after
// each record so that the scheduler's polling paths run.  Kernels are replaced
// by the CPU stand-ins of fake_kernels.cpp.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>

#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define HIP_SYMBOL(x) (&(x))

struct int2 {
    int x, y;
};

typedef enum {
    hipSuccess = 0,
    hipErrorOutOfMemory = 2,
    hipErrorInvalidValue = 1,
    hipErrorNotReady = 600,
} hipError_t;

typedef enum { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice,
               hipMemcpyDefault } hipMemcpyKind;
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };
typedef enum { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal } hipStreamCaptureMode;

struct FakeStream {
    int id;
};
struct FakeEvent {
    std::atomic<int> pending{0};  // queries left that report "not ready"
    std::atomic<uint64_t> seq{0};
};
typedef FakeStream *hipStream_t;
typedef FakeEvent *hipEvent_t;
typedef struct FakeGraph *hipGraph_t;
typedef struct FakeGraph *hipGraphExec_t;

struct hipDeviceProp_t {
    char gcnArchName[256];
    int multiProcessorCount;
};

// Every function below is defined in fake_hip.cpp.
hipError_t hipGetDeviceCount(int *n);
hipError_t hipSetDevice(int d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int d);
hipError_t hipMemGetInfo(size_t *freeb, size_t *total);
hipError_t hipMalloc(void **p, size_t n);
template <class T>
hipError_t hipMalloc(T **p, size_t n) { return hipMalloc(reinterpret_cast<void **>(p), n); }
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t n, unsigned flags);
template <class T>
hipError_t hipHostMalloc(T **p, size_t n, unsigned flags) { return hipHostMalloc(reinterpret_cast<void **>(p), n, flags); }
hipError_t hipHostFree(void *p);
hipError_t hipMallocAsync(void **p, size_t n, hipStream_t s);
hipError_t hipFreeAsync(void *p, hipStream_t s);
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, void *, char *, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);
