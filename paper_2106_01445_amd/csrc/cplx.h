// Small complex helpers (fp64) for the contour kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

__device__ __forceinline__ cplx cmk(double r, double i) { return cplx{r, i}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b)
{
    return cplx{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// a*b + c
__device__ __forceinline__ cplx cfma(cplx a, cplx b, cplx c)
{
    return cplx{fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
// c - a*b
__device__ __forceinline__ cplx cfnma(cplx a, cplx b, cplx c)
{
    return cplx{fma(-a.re, b.re, fma(a.im, b.im, c.re)), fma(-a.re, b.im, fma(-a.im, b.re, c.im))};
}
__device__ __forceinline__ cplx cscale(cplx a, double s) { return cplx{a.re * s, a.im * s}; }
__device__ __forceinline__ cplx crecip(cplx b)
{
    double d = 1.0 / fma(b.re, b.re, b.im * b.im);
    return cplx{b.re * d, -b.im * d};
}
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) { return cmul(a, crecip(b)); }
// principal square root
__device__ __forceinline__ cplx csqrt_p(cplx z)
{
    double r = hypot(z.re, z.im);
    double t = sqrt(0.5 * (fabs(z.re) + r));
    if (z.re >= 0.0) return cplx{t, z.im / (2.0 * t)};
    return cplx{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}
// principal logarithm
__device__ __forceinline__ cplx clog_p(cplx z) { return cplx{log(hypot(z.re, z.im)), atan2(z.im, z.re)}; }
__device__ __forceinline__ cplx cexp_(cplx z)
{
    double e = exp(z.re), s, c;
    sincos(z.im, &s, &c);
    return cplx{e * c, e * s};
}
