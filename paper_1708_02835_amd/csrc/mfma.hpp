// Matrix-core helpers for gfx950 (64-lane wavefronts).
//
// v_mfma_f64_16x16x4_f64 computes D(16×16) = A(16×4) · B(4×16) + C.  Lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; element r (0..3) of the
// per-lane result holds D[l / 16 + 4 r][l % 16] (rows interleaved by 4).
// The FP32 16x16x4 form takes operands the same way but returns
// D[4 (l / 16) + r][l % 16]; the BF16 16x16x32 form gives each lane 8
// consecutive k values, A[l % 16][8 (l / 16) + 0..7] and
// B[8 (l / 16) + 0..7][l % 16], with the FP32 result layout; the FP16
// 16x16x32 form takes the same layout.  These layouts are checked on the
// device by gl_selftest.
#pragma once

#include <hip/hip_runtime.h>

namespace gl {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));  // 16-byte vector loads and stores
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// result coordinates of element r of lane `lane`
__device__ inline int mfma_row(int lane, int r) { return (lane >> 4) + 4 * r; }  // FP64 form
__device__ inline int mfma_col(int lane) { return lane & 15; }
__device__ inline int mfma32_row(int lane, int r) { return 4 * (lane >> 4) + r; }  // FP32 / BF16 forms

__device__ inline d4 mfma_f64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline f4 mfma_f32(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ inline f4 mfma_bf16(bf16x8 a, bf16x8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline f4 mfma_f16(f16x8 a, f16x8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Value of v in lane l (l uniform across the wave), as two 32-bit readlanes.
__device__ inline double readlane_f64(double v, int l)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide sum (fixed butterfly order, identical on every lane).
__device__ inline double wave_sum(double v)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace gl
