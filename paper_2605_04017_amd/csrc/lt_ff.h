// Float-float ("double-float") arithmetic built from FP32 operations only.
// Every primitive disables floating-point contraction: fusing a product into
// a following sum (e.g. hi + lo of a TwoProduct into one FMA) would silently
// double-count the error term.
// A value is hi + lo with |lo| <= ulp(hi)/2.  The error-free transformations
// are Knuth's TwoSum, Dekker's Fast2Sum and the FMA-based TwoProduct; the
// compound operations follow the usual double-word algorithms (e.g. Joldes,
// Muller and Popescu, "Tight and rigorous error bounds for basic building
// blocks of double-word arithmetic", ACM TOMS 2017).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace lt {

struct ff {
    float h, l;
};

__host__ __device__ __forceinline__ ff ff_make(float h) {
#pragma clang fp contract(off)
    return ff{h, 0.0f};
}

// |a| >= |b|
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

__host__ __device__ __forceinline__ ff ff_add(ff x, ff y)
{
#pragma clang fp contract(off)
    ff s = two_sum(x.h, y.h);
    const ff t = two_sum(x.l, y.l);
    s.l += t.h;
    s = fast_two_sum(s.h, s.l);
    s.l += t.l;
    return fast_two_sum(s.h, s.l);
}

__host__ __device__ __forceinline__ ff ff_neg(ff x) {
#pragma clang fp contract(off)
    return ff{-x.h, -x.l};
}

__host__ __device__ __forceinline__ ff ff_sub(ff x, ff y) {
#pragma clang fp contract(off)
    return ff_add(x, ff_neg(y));
}

__host__ __device__ __forceinline__ ff ff_add_f(ff x, float b)
{
#pragma clang fp contract(off)
    const ff s = two_sum(x.h, b);
    return fast_two_sum(s.h, s.l + x.l);
}

__host__ __device__ __forceinline__ ff ff_mul(ff x, ff y)
{
#pragma clang fp contract(off)
    ff p = two_prod(x.h, y.h);
    p.l = fmaf(x.h, y.l, fmaf(x.l, y.h, p.l));
    return fast_two_sum(p.h, p.l);
}

__host__ __device__ __forceinline__ ff ff_mul_f(ff x, float b)
{
#pragma clang fp contract(off)
    ff p = two_prod(x.h, b);
    p.l = fmaf(x.l, b, p.l);
    return fast_two_sum(p.h, p.l);
}

__host__ __device__ __forceinline__ ff ff_sqr(ff x)
{
#pragma clang fp contract(off)
    ff p = two_prod(x.h, x.h);
    p.l = fmaf(2.0f * x.h, x.l, p.l);
    return fast_two_sum(p.h, p.l);
}

// x + a*b with a, b double-words (fused dot-product building block)
__host__ __device__ __forceinline__ ff ff_fma(ff a, ff b, ff x) {
#pragma clang fp contract(off)
    return ff_add(x, ff_mul(a, b));
}

__host__ __device__ __forceinline__ ff ff_div(ff x, ff y)
{
#pragma clang fp contract(off)
    const float q1 = x.h / y.h;
    // remainder x - q1*y in double-word
    const ff r = ff_sub(x, ff_mul_f(y, q1));
    const float q2 = r.h / y.h;
    return fast_two_sum(q1, q2);
}

__host__ __device__ __forceinline__ ff ff_sqrt(ff x)
{
#pragma clang fp contract(off)
    if (!(x.h > 0.0f))
        return ff{0.0f, 0.0f};
    const float s = sqrtf(x.h);
    // x - s^2, then one Newton correction
    const ff s2 = two_prod(s, s);
    const float r = ((x.h - s2.h) - s2.l) + x.l;
    return fast_two_sum(s, r / (2.0f * s));
}

__host__ __device__ __forceinline__ float ff_to_f(ff x) {
#pragma clang fp contract(off)
    return x.h + x.l;
}

}  // namespace lt
