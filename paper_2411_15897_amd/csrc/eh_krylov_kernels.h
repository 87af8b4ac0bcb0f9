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

// MODE 0: partial[i] = sum_p conj(V_i[p]) w[p]                   (i < m)
// MODE 1: w <- w - sum_i c_i V_i;  partial[i] = sum conj(V_i) w   (update + dot)
// MODE 2: w <- w - sum_i c_i V_i;  partial[0] = sum |w|^2          (update + norm)
// MODE 3: partial[0] = sum |w|^2
// MODE 4: partial[i] = sum conj(V_i) w and partial[m + i] = sum conj(V_i) V_{m-1}
//         (projections of w and the newest column of the Gram matrix V^H V)
// grid: (nblk, nrhs); block b owns the KRY_E * 256 entries starting at
// b * KRY_E * 256 (each thread KRY_E of them, 256 apart: coalesced).
// partial layout [r][blk][i] (i < m, or 1 for norms); coef layout [r][i].
constexpr int KRY_E = 4;
template <int MODE>
__global__ void __launch_bounds__(KRY_THREADS)
k_gs(int64_t n, int m, int nrhs, const c128* __restrict__ V, c128* __restrict__ w,
     const c128* __restrict__ coef, c128* __restrict__ partial) {
    __shared__ double lre[4][2 * KRY_MAXM], lim[4][2 * KRY_MAXM];
    const int r = blockIdx.y;
    const int nblk = gridDim.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * (KRY_E * KRY_THREADS) + threadIdx.x;
    c128* wr = w + (int64_t)r * n;
    c128 wv[KRY_E];
#pragma unroll
    for (int e = 0; e < KRY_E; ++e) {
        const int64_t p = base + e * KRY_THREADS;
        wv[e] = p < n ? wr[p] : mk(0.0, 0.0);
    }
    if (MODE == 1 || MODE == 2) {
        for (int t = 0; t < m; ++t) {
            const c128 cf = coef[r * m + t];
            const c128* Vt = V + ((int64_t)t * nrhs + r) * n;
#pragma unroll
            for (int e = 0; e < KRY_E; ++e) {
                const int64_t p = base + e * KRY_THREADS;
                if (p < n) wv[e] = wv[e] - cf * Vt[p];
            }
        }
#pragma unroll
        for (int e = 0; e < KRY_E; ++e) {
            const int64_t p = base + e * KRY_THREADS;
            if (p < n) wr[p] = wv[e];
        }
    }
    int mm = 1;
    if (MODE == 4) {
        mm = 2 * m;
        c128 vl[KRY_E];
        const c128* Vl = V + ((int64_t)(m - 1) * nrhs + r) * n;
#pragma unroll
        for (int e = 0; e < KRY_E; ++e) {
            const int64_t p = base + e * KRY_THREADS;
            vl[e] = p < n ? Vl[p] : mk(0.0, 0.0);
        }
        for (int t = 0; t < m; ++t) {
            const c128* Vt = V + ((int64_t)t * nrhs + r) * n;
            double ar = 0.0, ai = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
            for (int e = 0; e < KRY_E; ++e) {
                const int64_t p = base + e * KRY_THREADS;
                if (p < n) {
                    const c128 v = Vt[p];
                    ar += v.re * wv[e].re + v.im * wv[e].im;
                    ai += v.re * wv[e].im - v.im * wv[e].re;
                    gr += v.re * vl[e].re + v.im * vl[e].im;
                    gi += v.re * vl[e].im - v.im * vl[e].re;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                ar += __shfl_xor(ar, off, 64);
                ai += __shfl_xor(ai, off, 64);
                gr += __shfl_xor(gr, off, 64);
                gi += __shfl_xor(gi, off, 64);
            }
            if (lane == 0) {
                lre[wave][t] = ar; lim[wave][t] = ai;
                lre[wave][m + t] = gr; lim[wave][m + t] = gi;
            }
        }
    } else if (MODE == 0 || MODE == 1) {
        mm = m;
        for (int t = 0; t < m; ++t) {
            const c128* Vt = V + ((int64_t)t * nrhs + r) * n;
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int e = 0; e < KRY_E; ++e) {
                const int64_t p = base + e * KRY_THREADS;
                if (p < n) {
                    const c128 v = Vt[p];
                    ar += v.re * wv[e].re + v.im * wv[e].im;
                    ai += v.re * wv[e].im - v.im * wv[e].re;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                ar += __shfl_xor(ar, off, 64);
                ai += __shfl_xor(ai, off, 64);
            }
            if (lane == 0) { lre[wave][t] = ar; lim[wave][t] = ai; }
        }
    } else {
        double a = 0.0;
#pragma unroll
        for (int e = 0; e < KRY_E; ++e) a += wv[e].re * wv[e].re + wv[e].im * wv[e].im;
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        if (lane == 0) { lre[wave][0] = a; lim[wave][0] = 0.0; }
    }
    __syncthreads();
    if (threadIdx.x < mm) {
        const int t = threadIdx.x;
        const double sr = (lre[0][t] + lre[1][t]) + (lre[2][t] + lre[3][t]);
        const double si = (lim[0][t] + lim[1][t]) + (lim[2][t] + lim[3][t]);
        partial[((int64_t)r * nblk + blockIdx.x) * mm + t] = mk(sr, si);
    }
}

// out[r][i] = sum_blk partial[r][blk][i]: one block per (i, r), fixed-order
// tree, so the result does not depend on timing.
__global__ void __launch_bounds__(256)
k_reduce_partials(int nblk, int m, int nrhs, const c128* __restrict__ partial, c128* __restrict__ out) {
    __shared__ double sre[256], sim[256];
    const int i = blockIdx.x, r = blockIdx.y;
    double ar = 0.0, ai = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        const c128 v = partial[((int64_t)r * nblk + b) * m + i];
        ar += v.re; ai += v.im;
    }
    sre[threadIdx.x] = ar; sim[threadIdx.x] = ai;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sre[threadIdx.x] += sre[threadIdx.x + s];
            sim[threadIdx.x] += sim[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r * m + i] = mk(sre[0], sim[0]);
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

// out = value (graph-safe fill)
template <class V>
__global__ void __launch_bounds__(256)
k_fill(int64_t n, V* __restrict__ out, V value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) out[p] = value;
}

// dst[r * vd + q] = src[r * vs + q] for q < n, r < nrhs (graph-safe copy)
template <class V>
__global__ void __launch_bounds__(256)
k_copy_strided(int64_t n, int nrhs, const V* __restrict__ src, int64_t vs, V* __restrict__ dst, int64_t vd) {
    const int r = blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        dst[(int64_t)r * vd + q] = src[(int64_t)r * vs + q];
}

// out = a - b
__global__ void __launch_bounds__(256)
k_sub(int64_t n, const c128* __restrict__ a, const c128* __restrict__ b, c128* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
        out[p] = a[p] - b[p];
}

// x[r] += sum_{i < mcount} y[r][i] Z_i[r]   (Z in the multigrid precision;
// only the mcount columns built in this cycle are read -- later columns may
// hold stale or uninitialised data; y has row stride mstride)
template <class T>
__global__ void __launch_bounds__(256)
k_xupdate(int64_t n, int mcount, int mstride, int nrhs, const cplx<T>* __restrict__ Z,
          const c128* __restrict__ y, c128* __restrict__ x) {
    const int r = blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        c128 s = x[(int64_t)r * n + p];
        for (int i = 0; i < mcount; ++i)
            s = s + y[r * mstride + i] * ccast<double>(Z[((int64_t)i * nrhs + r) * n + p]);
        x[(int64_t)r * n + p] = s;
    }
}

}  // namespace eh
