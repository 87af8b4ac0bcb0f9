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
