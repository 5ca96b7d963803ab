// Device self-checks of the matrix-core lane layouts assumed by the kernels.
// Each probe feeds A[i][k] = i + 1 + 0.25 k... small exact values, lane by lane
// in the documented operand layout, and returns the raw per-lane results so
// the caller can compare them with D = A·B computed on the host.
#include "common.hpp"
#include "mfma.hpp"

namespace gl {

__device__ inline double probe_a(int i, int k) { return (double)(i + 1) + 0.25 * (double)k; }
__device__ inline double probe_b(int k, int j) { return (double)(2 * j - 7) - 0.5 * (double)k; }

__global__ void probe_f64(double *out)
{
    const int l = threadIdx.x;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    acc = mfma_f64(probe_a(l & 15, l >> 4), probe_b(l >> 4, l & 15), acc);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = acc[r];
}

__global__ void probe_f32(double *out)
{
    const int l = threadIdx.x;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma_f32((float)probe_a(l & 15, l >> 4), (float)probe_b(l >> 4, l & 15), acc);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = (double)acc[r];
}

__global__ void probe_bf16(double *out)
{
    const int l = threadIdx.x;
    bf16x8 a, b;
    for (int q = 0; q < 8; ++q) {
        const int k = 8 * (l >> 4) + q;
        a[q] = (__bf16)(float)((l & 15) + 1 + (k & 3));   // small integers: exact in bf16
        b[q] = (__bf16)(float)(((l & 15) % 5) - (k % 3));
    }
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma_bf16(a, b, acc);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = (double)acc[r];
}

__global__ void probe_f16(double *out)
{
    const int l = threadIdx.x;
    f16x8 a, b;
    for (int q = 0; q < 8; ++q) {
        const int k = 8 * (l >> 4) + q;
        a[q] = (_Float16)(float)((l & 15) + 1 + (k & 3));  // small integers: exact in fp16
        b[q] = (_Float16)(float)(((l & 15) % 5) - (k % 3));
    }
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma_f16(a, b, acc);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = (double)acc[r];
}

int selftest_mfma(int which, double *out_h, int64_t cap)
{
    double *d = nullptr;
    GL_HIP_TRY(hipMalloc(reinterpret_cast<void **>(&d), 256 * sizeof(double)));
    if (which == 0) probe_f64<<<1, 64>>>(d);
    else if (which == 1) probe_f32<<<1, 64>>>(d);
    else if (which == 2) probe_bf16<<<1, 64>>>(d);
    else probe_f16<<<1, 64>>>(d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(out_h, d, 256 * sizeof(double), hipMemcpyDeviceToHost);
    hipFree(d);
    if (e != hipSuccess) return gl_hip_fail(e, "selftest");
    (void)cap;
    return GL_OK;
}

}  // namespace gl
