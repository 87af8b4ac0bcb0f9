// Internal definitions shared by the kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eh {

// Interleaved complex number; alignment lets the compiler issue one 8- or
// 16-byte load per element.
template <class T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

using c64 = cplx<float>;
using c128 = cplx<double>;

template <class T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) { cplx<T> z; z.re = r; z.im = i; return z; }
template <class T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk<T>(a.re + b.re, a.im + b.im); }
template <class T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk<T>(a.re - b.re, a.im - b.im); }
template <class T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return mk<T>(s * a.re, s * a.im); }
template <class T>
__host__ __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return mk<T>(a.re, -a.im); }
template <class T>
__host__ __device__ __forceinline__ T cabs2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
// a / b (Smith-free: operands here are well scaled diagonal entries)
template <class T>
__host__ __device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
    T d = T(1) / (b.re * b.re + b.im * b.im);
    return mk<T>((a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d);
}
// conj(a) * b
template <class T>
__host__ __device__ __forceinline__ cplx<T> cdotc(cplx<T> a, cplx<T> b) {
    return mk<T>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <class To, class Ti>
__host__ __device__ __forceinline__ cplx<To> ccast(cplx<Ti> a) { return mk<To>(To(a.re), To(a.im)); }

template <class T>
__host__ __device__ __forceinline__ cplx<T> czero() { return mk<T>(T(0), T(0)); }

__host__ __device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc + a * b as four explicit fused multiply-adds in a fixed order.  The
// compiler's own contraction of acc + (a * b) depends on the surrounding
// code (how often each product is used), so the same stencil could round
// differently in two inlined copies; fixed fmas give the same bits wherever
// this is inlined, in four instructions instead of six.
template <class T>
__host__ __device__ __forceinline__ cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> acc) {
    return mk<T>(fmat(-a.im, b.im, fmat(a.re, b.re, acc.re)), fmat(a.im, b.re, fmat(a.re, b.im, acc.im)));
}

// Grid of points of one block on one level: extents per axis (x first).
struct Dims {
    int g[3];
    __host__ __device__ int64_t np() const { return (int64_t)g[0] * g[1] * g[2]; }
};

// Stencil half widths per axis and the number of stored offsets.
struct Widths {
    int w[3];
    __host__ __device__ int nst() const { return (2 * w[0] + 1) * (2 * w[1] + 1) * (2 * w[2] + 1); }
};

}  // namespace eh
