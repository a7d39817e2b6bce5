// Double-word ("float-float") arithmetic built from FP32 operations only.
// A value is h + l.  Every primitive disables floating-point contraction:
// fusing a product into a following sum (e.g. h + l of a TwoProduct into one
// FMA) would silently double-count the error term.
//
// The error-free transformations are Knuth's TwoSum, Dekker's Fast2Sum and
// the FMA-based TwoProduct.  The compound operations are the cheap forms of
// the usual double-word algorithms (Joldes, Muller and Popescu, "Tight and
// rigorous error bounds for basic building blocks of double-word
// arithmetic", ACM TOMS 2017):
//   - dw_add is the "sloppy" sum: one TwoSum of the leading words, the
//     trailing words added in FP32, no renormalisation.  Its absolute error
//     is about 2u^2 (|x| + |y|) with u = 2^-24; only its relative error grows
//     under cancellation, and the tracer needs absolute accuracy.
//   - dw_mul is TwoProduct of the leading words plus the two cross terms,
//     without renormalisation (error about 3u^2 |x y|).
//   - Results are therefore unnormalised: |l| may exceed half an ulp of h
//     after a cancelling sum.  dw_norm (Fast2Sum) restores the invariant;
//     the tracer renormalises its carried state once per interaction.
//   - dw_div and dw_sqrt take their first approximation from the hardware
//     reciprocal and square root (about one ulp, not correctly rounded) and
//     add one remainder correction.  The correction's error is quadratic in
//     the first term's relative error, so both renormalise the divisor and
//     the radicand first: from an unnormalised operand the first term would
//     start |l/h| off instead of one ulp.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace lt {

struct ff {
    float h, l;
};

#ifndef __HIP_DEVICE_COMPILE__
// Host builds stand in for the hardware instructions with correctly rounded
// results; an error-budget build (-DLT_HOST_APPROX_ULP=+1 or -1) moves them
// one ulp up or down to model the hardware's error.
__host__ __forceinline__ float host_ulp_error(float v)
{
#ifdef LT_HOST_APPROX_ULP
    return nextafterf(v, LT_HOST_APPROX_ULP > 0 ? INFINITY : -INFINITY);
#else
    return v;
#endif
}
#endif

// Approximate 1/x and sqrt(x) (about one ulp) for first terms that a
// correction follows, and for quantities needed only to FP32 accuracy.  On
// the device each is one hardware instruction (v_rcp_f32, v_sqrt_f32).
__host__ __device__ __forceinline__ float approx_rcp(float x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(x);
#else
    return host_ulp_error(1.0f / x);
#endif
}

__host__ __device__ __forceinline__ float approx_sqrt(float x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_sqrtf(x);
#else
    return host_ulp_error(sqrtf(x));
#endif
}

__host__ __device__ __forceinline__ ff ff_make(float h) { return ff{h, 0.0f}; }

__host__ __device__ __forceinline__ ff ff_neg(ff x) { return ff{-x.h, -x.l}; }

// 2x, exact
__host__ __device__ __forceinline__ ff ff_twice(ff x) {
#pragma clang fp contract(off)
    return ff{x.h + x.h, x.l + x.l};
}

// |a| >= |b| (or a == 0)
__host__ __device__ __forceinline__ ff fast_two_sum(float a, float b)
{
#pragma clang fp contract(off)
    const float s = a + b;
    return ff{s, b - (s - a)};
}

__host__ __device__ __forceinline__ ff two_sum(float a, float b)
{
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    return ff{s, (a - (s - bb)) + (b - bb)};
}

__host__ __device__ __forceinline__ ff two_prod(float a, float b)
{
#pragma clang fp contract(off)
    const float p = a * b;
    return ff{p, fmaf(a, b, -p)};
}

__host__ __device__ __forceinline__ ff dw_norm(ff x) { return fast_two_sum(x.h, x.l); }

__host__ __device__ __forceinline__ ff dw_add(ff x, ff y)
{
#pragma clang fp contract(off)
    const ff s = two_sum(x.h, y.h);
    return ff{s.h, (x.l + y.l) + s.l};
}

__host__ __device__ __forceinline__ ff dw_sub(ff x, ff y) { return dw_add(x, ff_neg(y)); }

__host__ __device__ __forceinline__ ff dw_add_f(ff x, float b)
{
#pragma clang fp contract(off)
    const ff s = two_sum(x.h, b);
    return ff{s.h, x.l + s.l};
}

__host__ __device__ __forceinline__ ff dw_mul(ff x, ff y)
{
#pragma clang fp contract(off)
    const float p = x.h * y.h;
    return ff{p, fmaf(x.h, y.l, fmaf(x.l, y.h, fmaf(x.h, y.h, -p)))};
}

__host__ __device__ __forceinline__ ff dw_mul_f(ff x, float b)
{
#pragma clang fp contract(off)
    const float p = x.h * b;
    return ff{p, fmaf(x.l, b, fmaf(x.h, b, -p))};
}

__host__ __device__ __forceinline__ ff dw_sqr(ff x)
{
#pragma clang fp contract(off)
    const float p = x.h * x.h;
    return ff{p, fmaf(x.h + x.h, x.l, fmaf(x.h, x.h, -p))};
}

// x / y: q1 = x_h / y_h from the approximate reciprocal, then the remainder
// x - q1 y (its leading part x_h - q1 y_h is exact by Sterbenz's lemma, as
// q1 y_h lies within a few ulps of x_h) divided the same way.
__host__ __device__ __forceinline__ ff dw_div(ff x, ff y)
{
#pragma clang fp contract(off)
    y = dw_norm(y);
    const float r = approx_rcp(y.h);
    const float q1 = x.h * r;
    const float p = q1 * y.h;
    const float e = fmaf(q1, y.h, -p);
    const float rem = fmaf(-q1, y.l, ((x.h - p) - e) + x.l);
    return ff{q1, rem * r};
}

// sqrt(x) for x > 0 (0 otherwise): s from the approximate root, then one
// Newton correction (x - s^2) / 2s.
__host__ __device__ __forceinline__ ff dw_sqrt(ff x)
{
#pragma clang fp contract(off)
    x = dw_norm(x);
    if (!(x.h > 0.0f))
        return ff{0.0f, 0.0f};
    const float s = approx_sqrt(x.h);
    const float rem = fmaf(-s, s, x.h) + x.l;
    return ff{s, rem * (0.5f * approx_rcp(s))};
}

__host__ __device__ __forceinline__ float ff_to_f(ff x) {
#pragma clang fp contract(off)
    return x.h + x.l;
}

}  // namespace lt
