// Double-double arithmetic for the exact path and the model build.
//
// A value is hi + lo with |lo| <= ulp(hi)/2, ~106 significant bits.  Built from
// two error-free transformations: Knuth's TwoSum (s + e = a + b exactly) and
// the product with its rounding error recovered by one fused multiply-add
// (Dekker 1971 with an FMA in place of the splitting).  Division and square
// root take an fp64 estimate and one Newton correction in double-double.
// exp uses argument reduction by ln 2, a further halving, a Taylor series and
// repeated squaring.  Every function turns floating-point contraction off: a
// product fused into a later addition would break the error-free steps.
#pragma once
#include <hip/hip_runtime.h>

struct dd {
    double hi, lo;
};

__host__ __device__ __forceinline__ dd dd_make(double a)
{
#pragma clang fp contract(off)
    return dd{a, 0.0};
}

__host__ __device__ __forceinline__ dd two_sum(double a, double b)
{
#pragma clang fp contract(off)
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd{s, e};
}

__host__ __device__ __forceinline__ dd quick_two_sum(double a, double b)
{
#pragma clang fp contract(off)
    double s = a + b;
    return dd{s, b - (s - a)};
}

__host__ __device__ __forceinline__ dd two_prod(double a, double b)
{
#pragma clang fp contract(off)
    double p = a * b;
    return dd{p, fma(a, b, -p)};
}

__host__ __device__ __forceinline__ dd dd_add(dd x, dd y)
{
#pragma clang fp contract(off)
    dd s = two_sum(x.hi, y.hi);
    dd t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__host__ __device__ __forceinline__ dd dd_neg(dd x)
{
#pragma clang fp contract(off)
    return dd{-x.hi, -x.lo};
}
__host__ __device__ __forceinline__ dd dd_sub(dd x, dd y)
{
#pragma clang fp contract(off)
    return dd_add(x, dd_neg(y));
}

__host__ __device__ __forceinline__ dd dd_add_d(dd x, double b)
{
#pragma clang fp contract(off)
    dd s = two_sum(x.hi, b);
    s.lo += x.lo;
    return quick_two_sum(s.hi, s.lo);
}

__host__ __device__ __forceinline__ dd dd_mul(dd x, dd y)
{
#pragma clang fp contract(off)
    dd p = two_prod(x.hi, y.hi);
    p.lo = fma(x.hi, y.lo, p.lo);
    p.lo = fma(x.lo, y.hi, p.lo);
    return quick_two_sum(p.hi, p.lo);
}

__host__ __device__ __forceinline__ dd dd_mul_d(dd x, double b)
{
#pragma clang fp contract(off)
    dd p = two_prod(x.hi, b);
    p.lo = fma(x.lo, b, p.lo);
    return quick_two_sum(p.hi, p.lo);
}

// x - y*z
__host__ __device__ __forceinline__ dd dd_fnma(dd x, dd y, dd z)
{
#pragma clang fp contract(off)
    return dd_sub(x, dd_mul(y, z));
}

__host__ __device__ __forceinline__ dd dd_div(dd x, dd y)
{
#pragma clang fp contract(off)
    double q1 = x.hi / y.hi;
    dd r = dd_sub(x, dd_mul_d(y, q1));
    double q2 = r.hi / y.hi;
    r = dd_sub(r, dd_mul_d(y, q2));
    double q3 = r.hi / y.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add_d(q, q3);
}

__host__ __device__ __forceinline__ dd dd_recip(dd y)
{
#pragma clang fp contract(off)
    return dd_div(dd_make(1.0), y);
}

// x / b for an fp64 divisor
__host__ __device__ __forceinline__ dd dd_div_d(dd x, double b)
{
#pragma clang fp contract(off)
    double q1 = x.hi / b;
    dd r = dd_sub(x, two_prod(q1, b));
    double q2 = r.hi / b;
    r = dd_sub(r, two_prod(q2, b));
    double q3 = r.hi / b;
    return dd_add_d(quick_two_sum(q1, q2), q3);
}

// sqrt for x > 0: s = sqrt(hi), then s + (x - s^2) / (2 s).
__host__ __device__ __forceinline__ dd dd_sqrt(dd x)
{
#pragma clang fp contract(off)
    double s = sqrt(x.hi);
    dd s2 = two_prod(s, s);
    dd r = dd_sub(x, s2);
    return quick_two_sum(s, r.hi / (2.0 * s));
}

// 1/sqrt(x) for x > 0, refined by one Newton step y <- y + y (1 - x y^2) / 2.
__host__ __device__ __forceinline__ dd dd_rsqrt(dd x)
{
#pragma clang fp contract(off)
    double y0 = 1.0 / sqrt(x.hi);
    dd y = dd_make(y0);
    dd e = dd_sub(dd_make(1.0), dd_mul(x, dd_mul(y, y)));
    y = dd_add(y, dd_mul_d(dd_mul(y, e), 0.5));
    e = dd_sub(dd_make(1.0), dd_mul(x, dd_mul(y, y)));
    return dd_add(y, dd_mul_d(dd_mul(y, e), 0.5));
}

// exp(x) for |x| < 700.  x = k ln2 + r; r' = r / 1024; Taylor to degree 14;
// square 10 times; scale by 2^k.
__host__ __device__ inline dd dd_exp(dd x)
{
#pragma clang fp contract(off)
    const dd ln2 = dd{6.93147180559945286227e-01, 2.31904681384629955842e-17};
    double k = rint(x.hi / ln2.hi);
    dd r = dd_sub(x, dd_mul_d(ln2, k));
    r = dd_mul_d(r, 1.0 / 1024.0);
    // Horner: sum_{i=0}^{14} r^i / i!
    dd s = dd_make(1.0);
    for (int i = 14; i >= 1; --i) {
        s = dd_div_d(dd_mul(s, r), (double)i);  // s = 1 + s * r / i
        s = dd_add_d(s, 1.0);
    }
    // s now holds 1 + r(1 + r/2(1 + r/3(...))) = exp(r)
    for (int i = 0; i < 10; ++i) s = dd_mul(s, s);
    double sc = ldexp(1.0, (int)k);
    return dd{s.hi * sc, s.lo * sc};
}
