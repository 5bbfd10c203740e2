// Device helpers shared by the HIP kernels of libscocg (not part of the C ABI).
#pragma once
#include "scocg_internal.h"

// No implicit contraction: every fused multiply-add is written out, so the arithmetic
// (and its rounding) is the same in every template instance.
#pragma clang fp contract(off)

namespace scocg {

static constexpr int WG = 256;

// a * b + c with explicit fused multiply-adds
__device__ inline double2 cfma(double2 a, double2 b, double2 c)
{
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ inline float2 cfma(float2 a, float2 b, float2 c)
{
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
__device__ inline double rfma(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float rfma(float a, float b, float c) { return fmaf(a, b, c); }

template <typename V>
__device__ inline V to_v(double2 a);
template <>
__device__ inline double2 to_v<double2>(double2 a) { return a; }
template <>
__device__ inline float2 to_v<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }

}  // namespace scocg
