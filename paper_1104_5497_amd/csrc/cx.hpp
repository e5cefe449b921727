// cx.hpp -- minimal complex arithmetic on a real type T (float or double),
// usable in device code and, for host-side checks, in host code.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#ifndef NPHC_HD
#define NPHC_HD __host__ __device__ __forceinline__
#endif

// Keeps the instruction scheduler from interleaving the phases on either side
// (device code only), which bounds the number of values live at once.
#if defined(__HIP_DEVICE_COMPILE__)
#define NPHC_PHASE() __builtin_amdgcn_sched_barrier(0)
#else
#define NPHC_PHASE() ((void)0)
#endif

// Read-only data that no kernel writes while it is read (the couplings): the
// constant address space lets wave-uniform reads use scalar loads into SGPRs
// instead of vector loads into VGPRs.  Divergent addresses still work (they
// become vector loads).
#ifndef NPHC_RO
#if defined(__HIP_DEVICE_COMPILE__)
#define NPHC_RO __attribute__((address_space(4)))
#else
#define NPHC_RO
#endif
#endif

namespace nphc {

template <class T>
struct cx {
    T re, im;
};

template <class T> __host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {s * a.re, s * a.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <class T> __host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <class T> __host__ __device__ __forceinline__ T abs1(cx<T> a) { return fabs(a.re) + fabs(a.im); }
template <class T> __host__ __device__ __forceinline__ T absmax(cx<T> a) { return fmax(fabs(a.re), fabs(a.im)); }
template <class T> __host__ __device__ __forceinline__ cx<T> sel(bool c, cx<T> a, cx<T> b) { return c ? a : b; }

// c - a * b
template <class T> __host__ __device__ __forceinline__ cx<T> fnma(cx<T> a, cx<T> b, cx<T> c)
{
    return {c.re - a.re * b.re + a.im * b.im, c.im - a.re * b.im - a.im * b.re};
}
// c + a * b
template <class T> __host__ __device__ __forceinline__ cx<T> fma(cx<T> a, cx<T> b, cx<T> c)
{
    return {c.re + a.re * b.re - a.im * b.im, c.im + a.re * b.im + a.im * b.re};
}

// y + a x for a real scalar a
template <class T> __host__ __device__ __forceinline__ cx<T> axpy(T a, cx<T> x, cx<T> y)
{
    return {y.re + a * x.re, y.im + a * x.im};
}

// Reciprocal of a real number: the hardware reciprocal (1 ulp) in float32;
// in float64 the hardware estimate refined by two Newton steps.
__host__ __device__ __forceinline__ float rrcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ double rrcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

// 1 / a, scaled by the larger component so that |a|^2 neither overflows nor
// underflows for any finite nonzero a.
template <class T> __host__ __device__ __forceinline__ cx<T> rcp(cx<T> a)
{
    T s = absmax(a);
    T inv_s = rrcp(s);
    T ar = a.re * inv_s, ai = a.im * inv_s;
    T d = rrcp((ar * ar + ai * ai) * s);
    return {ar * d, -ai * d};
}

// principal square root
template <class T> __host__ __device__ __forceinline__ cx<T> csqrt(cx<T> a)
{
    T r = sqrt(sqrt(a.re * a.re + a.im * a.im) * T(0.5) + fabs(a.re) * T(0.5));
    if (r == T(0)) return {T(0), T(0)};
    T q = a.im / (T(2) * r);
    if (a.re >= T(0)) return {r, q};
    return {fabs(q), a.im >= T(0) ? r : -r};
}

}  // namespace nphc
