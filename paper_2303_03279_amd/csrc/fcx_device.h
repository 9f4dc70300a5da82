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

__device__ __forceinline__ int sgn_of(double v) { return (v > 0.0) - (v < 0.0); }

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T> __device__ __forceinline__ T sqrt_ratio(double r);
template <> __device__ __forceinline__ float sqrt_ratio<float>(double r) { return sqrtf((float)r); }
template <> __device__ __forceinline__ double sqrt_ratio<double>(double r) { return sqrt(r); }

__device__ __forceinline__ bool finite_v(float v) { return isfinite(v); }
__device__ __forceinline__ bool finite_v(double v) { return isfinite(v); }

// num / den for a metric in [-1, 1]: FP64 operands of any scale are brought
// to den in [0.5, 1) by an exact power-of-two scaling, then divided in FP32
// (the FP64 instantiation divides in FP64)
template <typename T> __device__ __forceinline__ T ratio_t(double num, double den);
template <> __device__ __forceinline__ float ratio_t<float>(double num, double den)
{
    int e;
    const double dm = frexp(den, &e);
    return __fdividef((float)ldexp(num, -e), (float)dm);
}
template <> __device__ __forceinline__ double ratio_t<double>(double num, double den) { return num / den; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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
