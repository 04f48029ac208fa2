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

// fp32 complex, for the cluster eliminations of the mixed-precision tier
struct alignas(8) cplxf {
    float re, im;
};
__device__ __forceinline__ cplxf cmkf(float r, float i) { return cplxf{r, i}; }
__device__ __forceinline__ cplxf cadd(cplxf a, cplxf b) { return cplxf{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplxf csub(cplxf a, cplxf b) { return cplxf{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplxf cmul(cplxf a, cplxf b)
{
    return cplxf{fmaf(a.re, b.re, -a.im * b.im), fmaf(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplxf cfma(cplxf a, cplxf b, cplxf c)
{
    return cplxf{fmaf(a.re, b.re, fmaf(-a.im, b.im, c.re)), fmaf(a.re, b.im, fmaf(a.im, b.re, c.im))};
}
__device__ __forceinline__ cplxf cfnma(cplxf a, cplxf b, cplxf c)
{
    return cplxf{fmaf(-a.re, b.re, fmaf(a.im, b.im, c.re)), fmaf(-a.re, b.im, fmaf(-a.im, b.re, c.im))};
}
__device__ __forceinline__ cplx to_d(cplx a) { return a; }
__device__ __forceinline__ cplx to_d(cplxf a) { return cplx{(double)a.re, (double)a.im}; }
template <class C> __device__ __forceinline__ C from_d(cplx a);
template <> __device__ __forceinline__ cplx from_d<cplx>(cplx a) { return a; }
template <> __device__ __forceinline__ cplxf from_d<cplxf>(cplx a) { return cplxf{(float)a.re, (float)a.im}; }
__device__ __forceinline__ cplx cneg(cplx a) { return cplx{-a.re, -a.im}; }
__device__ __forceinline__ cplxf cneg(cplxf a) { return cplxf{-a.re, -a.im}; }
