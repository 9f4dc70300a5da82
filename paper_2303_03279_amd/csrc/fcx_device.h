// Device helpers shared by the HIP kernel files.
#pragma once

#include <math.h>

#include "fcx_internal.h"

#pragma clang fp contract(off)

namespace fcx {

template <typename T> struct V2;
template <> struct V2<float> { typedef float2 t; };
template <> struct V2<double> { typedef double2 t; };

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Raw buffer access (vector memory instructions through a buffer resource):
// a uniform base and byte range in scalar registers, a 32-bit per-lane byte
// offset.  An offset outside the range reads 0 and drops the store.
typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int RSRC_WORD3 = 0x00020000;   // untyped 32-bit data, gfx9 family
// Cache policy of the buffer accesses (the pair-state planes): the
// non-temporal hint (bit 1).  Every state element is read and written once
// per push, so marking those lines for early eviction keeps the operands that
// are reused across workgroups (ring spectra, z-scored samples) in L2 and the
// MALL.  Measured on the 5000-node all-8 push: 3.10 -> 2.76 ms, bit-identical.
constexpr int PLANE_AUX = 2;

// base and bytes must be uniform; they are read from the first lane so the
// resource always lives in scalar registers
__device__ __forceinline__ Rsrc tile_rsrc(void *base, uint32_t bytes)
{
    const uint64_t a = (uint64_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    void *ub = (void *)(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), RSRC_WORD3);
}
__device__ __forceinline__ double buf_ld_f64(Rsrc r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, PLANE_AUX));
}
__device__ __forceinline__ void buf_st_f64(Rsrc r, uint32_t off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, PLANE_AUX);
}
__device__ __forceinline__ int buf_ld_i32(Rsrc r, uint32_t off)
{
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, PLANE_AUX);
}
__device__ __forceinline__ void buf_st_i32(Rsrc r, uint32_t off, int v)
{
    __builtin_amdgcn_raw_buffer_store_b32((unsigned)v, r, off, 0, PLANE_AUX);
}
__device__ __forceinline__ int buf_ld_i8(Rsrc r, uint32_t off)
{
    return (int)(signed char)__builtin_amdgcn_raw_buffer_load_b8(r, off, 0, PLANE_AUX);
}
__device__ __forceinline__ void buf_st_i8(Rsrc r, uint32_t off, int v)
{
    __builtin_amdgcn_raw_buffer_store_b8((unsigned char)v, r, off, 0, PLANE_AUX);
}
__device__ __forceinline__ int buf_ld_i16(Rsrc r, uint32_t off)
{
    return (int)(short)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, PLANE_AUX);
}
__device__ __forceinline__ void buf_st_i16(Rsrc r, uint32_t off, int v)
{
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, off, 0, PLANE_AUX);
}

__device__ __forceinline__ int sgn_of(double v) { return (v > 0.0) - (v < 0.0); }

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Finalisation arithmetic of a metric in [-1, 1] (or [0, 1]) in the
// session's precision.  FP32 uses the hardware square root and reciprocal
// (about 1 ulp, far inside the 1e-5 metric tolerance) instead of the
// correctly rounded library sequences; FP64 stays exact IEEE.
template <typename T> __device__ __forceinline__ T sqrt_t(T v);
template <> __device__ __forceinline__ float sqrt_t<float>(float v) { return __builtin_amdgcn_sqrtf(v); }
template <> __device__ __forceinline__ double sqrt_t<double>(double v) { return sqrt(v); }

// 1/sqrt(x) of an FP64 x > 0 feeding an FP32 session's unit phasor: the
// hardware estimate (no Newton step) is far finer than the phasor's FP32
// rounding; FP64 sessions keep the refined library value.
template <typename T> __device__ __forceinline__ double rsqrt_t(double x);
template <> __device__ __forceinline__ double rsqrt_t<float>(double x) { return __builtin_amdgcn_rsq(x); }
template <> __device__ __forceinline__ double rsqrt_t<double>(double x) { return rsqrt(x); }

template <typename T> __device__ __forceinline__ T sqrt_ratio(double r);
template <> __device__ __forceinline__ float sqrt_ratio<float>(double r) { return __builtin_amdgcn_sqrtf((float)r); }
template <> __device__ __forceinline__ double sqrt_ratio<double>(double r) { return sqrt(r); }

__device__ __forceinline__ bool finite_v(float v) { return isfinite(v); }
__device__ __forceinline__ bool finite_v(double v) { return isfinite(v); }

// num / den: FP64 operands of any scale are brought to den in [0.5, 1) by an
// exact power-of-two scaling, then the FP32 quotient is num * rcp(den) (the
// FP64 instantiation divides in FP64)
template <typename T> __device__ __forceinline__ T ratio_t(double num, double den);
template <> __device__ __forceinline__ float ratio_t<float>(double num, double den)
{
    int e;
    const double dm = frexp(den, &e);
    return (float)ldexp(num, -e) * __builtin_amdgcn_rcpf((float)dm);
}
template <> __device__ __forceinline__ double ratio_t<double>(double num, double den) { return num / den; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Im(a conj b) of two FP32 values in FP64: both products are exact in FP64,
// so the result is the correctly rounded value of the exact difference, an
// exact zero included.  The first product enters as fma(-a.x, b.y, +0), which
// is never -0, so the result is never -0 either.
__device__ __forceinline__ double im_cross(float2 a, double bx, double by)
{
    return __builtin_fma((double)a.y, bx, __builtin_fma(-(double)a.x, by, 0.0));
}

// sign of an FP64 value that is not -0, as -1, 0 or 1 in one vector
// operation: its high word read as a signed integer is positive, zero or
// negative with it (a nonzero product difference of FP32 values is at least
// 2^-298, so its high word is never 0), clamped to [-1, 1] (an integer median)
__device__ __forceinline__ int sign_of_f64(double v)
{
    int r;
    asm("v_med3_i32 %0, %1, -1, 1" : "=v"(r) : "v"(__double2hiint(v)));
    return r;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  This bijection on [0, n) gives the workgroups of one XCD a contiguous
// run of work items, so neighbouring items (slices of one tile, tiles of one
// row) share that XCD's L2.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_item(int b, int n)
{
    const int q = n / NUM_XCD, rem = n % NUM_XCD;
    const int x = b % NUM_XCD, r = b / NUM_XCD;
    return x * q + min(x, rem) + r;
}

}  // namespace fcx
