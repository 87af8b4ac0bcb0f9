// FP64 reductions and vector updates of the flexible GMRES Arnoldi process
// (classical Gram-Schmidt applied twice).  Reductions are deterministic:
// every block writes its partial sums, a second kernel adds them in a fixed
// order, so FP64 runs are bitwise repeatable.
//
// Basis layout: vector i of right-hand side r starts at V + (i*nrhs + r)*n.
#pragma once

#include "eh_common.h"

namespace eh {

constexpr int KRY_THREADS = 256;
constexpr int KRY_MAXM = 32;   // columns handled by one pass

// Block-wide sum of a double across 256 threads (4 wavefronts).
__device__ __forceinline__ double block_sum(double v, double* lds) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = lds[0] + lds[1] + lds[2] + lds[3];
    return s;
}

// MODE 0: partial[i] = sum_p conj(V_i[p]) w[p]                   (i < m)
// MODE 1: w <- w - sum_i c_i V_i;  partial[i] = sum conj(V_i) w   (update + dot)
// MODE 2: w <- w - sum_i c_i V_i;  partial[0] = sum |w|^2          (update + norm)
// MODE 3: partial[0] = sum |w|^2
// grid: (nblk, nrhs); partial layout [r][blk][i] (i < m, or 1 for norms).
// coef layout [r][i] (device).
template <int MODE>
__global__ void __launch_bounds__(KRY_THREADS)
k_gs(int64_t n, int m, int nrhs, const c128* __restrict__ V, c128* __restrict__ w,
     const c128* __restrict__ coef, c128* __restrict__ partial) {
    __shared__ double lds[4];
    const int r = blockIdx.y;
    const int nblk = gridDim.x;
    c128* wr = w + (int64_t)r * n;
    double accr[KRY_MAXM], acci[KRY_MAXM];
    c128 cf[KRY_MAXM];
#pragma unroll
    for (int t = 0; t < KRY_MAXM; ++t) {
        accr[t] = 0.0; acci[t] = 0.0;
        cf[t] = (MODE == 1 || MODE == 2) && t < m ? coef[r * m + t] : mk(0.0, 0.0);
    }
    const int64_t stride = (int64_t)nblk * KRY_THREADS;
    for (int64_t p = (int64_t)blockIdx.x * KRY_THREADS + threadIdx.x; p < n; p += stride) {
        c128 wv = wr[p];
        if (MODE == 1 || MODE == 2) {
#pragma unroll
            for (int t = 0; t < KRY_MAXM; ++t) {
                if (t < m) wv = wv - cf[t] * V[((int64_t)t * nrhs + r) * n + p];
            }
            wr[p] = wv;
        }
        if (MODE == 0 || MODE == 1) {
#pragma unroll
            for (int t = 0; t < KRY_MAXM; ++t) {
                if (t < m) {
                    const c128 v = V[((int64_t)t * nrhs + r) * n + p];
                    accr[t] += v.re * wv.re + v.im * wv.im;
                    acci[t] += v.re * wv.im - v.im * wv.re;
                }
            }
        } else {
            accr[0] += wv.re * wv.re + wv.im * wv.im;
        }
    }
    const int mm = (MODE == 0 || MODE == 1) ? m : 1;
    for (int t = 0; t < mm; ++t) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int q = 0; q < KRY_MAXM; ++q) if (q == t) { sr = accr[q]; si = acci[q]; }
        sr = block_sum(sr, lds);
        si = block_sum(si, lds);
        if (threadIdx.x == 0) partial[((int64_t)r * nblk + blockIdx.x) * mm + t] = mk(sr, si);
    }
}

// out[r][i] = sum_blk partial[r][blk][i] in block order; also out2 = out
// accumulated into acc[r][i] when acc != nullptr.
__global__ void k_reduce_partials(int nblk, int m, int nrhs, const c128* __restrict__ partial,
                                  c128* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrhs * m) return;
    const int r = t / m, i = t % m;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const c128 v = partial[((int64_t)r * nblk + b) * m + i];
        sr += v.re; si += v.im;
    }
    out[t] = mk(sr, si);
}

// v[r] = s[r] * w[r]
__global__ void __launch_bounds__(256)
k_scale(int64_t n, int nrhs, const double* __restrict__ s, const c128* __restrict__ w,
        c128* __restrict__ v) {
    const int r = blockIdx.y;
    const double sc = s[r];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
        v[(int64_t)r * n + p] = sc * w[(int64_t)r * n + p];
}

// out = a - b
__global__ void __launch_bounds__(256)
k_sub(int64_t n, const c128* __restrict__ a, const c128* __restrict__ b, c128* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
        out[p] = a[p] - b[p];
}

// x[r] += sum_i y[r][i] Z_i[r]   (Z in the multigrid precision)
template <class T>
__global__ void __launch_bounds__(256)
k_xupdate(int64_t n, int m, int nrhs, const cplx<T>* __restrict__ Z, const c128* __restrict__ y,
          c128* __restrict__ x) {
    const int r = blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        c128 s = x[(int64_t)r * n + p];
        for (int i = 0; i < m; ++i)
            s = s + y[r * m + i] * ccast<double>(Z[((int64_t)i * nrhs + r) * n + p]);
        x[(int64_t)r * n + p] = s;
    }
}

}  // namespace eh
