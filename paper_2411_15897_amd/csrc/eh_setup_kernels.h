// Setup kernels (FP64, run once per context):
//  k_galerkin       coarse stencil of X_H = R X_h P (eq. galerkin) in stencil
//                   form, one thread per coarse point;
//  k_dense_from_stencil / Gauss-Jordan kernels: explicit inverse of the
//                   coarsest operator with partial pivoting, applied later
//                   as a dense matrix (the paper's direct coarsest solve).
#pragma once

#include "eh_common.h"
#include "eh_mg_kernels.h"

namespace eh {

constexpr int GAL_MAXW = 2;                                  // coarse half width
constexpr int GAL_MAXN = (2 * GAL_MAXW + 1) * (2 * GAL_MAXW + 1) * (2 * GAL_MAXW + 1);

// Fine stencil (widths wf, fine grid df) -> coarse stencil (widths wc,
// coarse grid dc).  For coarse point I: sum over fine k in the support of
// row I of R, over fine offsets o, over coarse parents J of l = k + o.
__global__ void __launch_bounds__(64)
k_galerkin(Dims df, Widths wf, const c128* __restrict__ cf, Dims dc, Widths wc, int nodal_mask, int mixed,
           c128* __restrict__ cc, int* __restrict__ overflow) {
    const int64_t npc = dc.np();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npc) return;
    const int I = (int)(q % dc.g[0]);
    const int J = (int)((q / dc.g[0]) % dc.g[1]);
    const int K = (int)(q / ((int64_t)dc.g[0] * dc.g[1]));
    c128 acc[GAL_MAXN];
    const int ncs = wc.nst();
    for (int t = 0; t < ncs; ++t) acc[t] = mk(0.0, 0.0);
    const bool nz = (nodal_mask & 4) != 0;
    const bool three = (df.g[2] > 1) || nz;
    Transfer1D rx, ry, rz;
    rx.restrict_support(I, nodal_mask & 1, df.g[0], mixed);
    ry.restrict_support(J, nodal_mask & 2, df.g[1], mixed);
    if (three) rz.restrict_support(K, nz, df.g[2], mixed);
    else { rz.n = 1; rz.idx[0] = 0; rz.wt[0] = 1.0f; }
    const int64_t npf = df.np();
    const int NXf = 2 * wf.w[0] + 1, NYf = 2 * wf.w[1] + 1;
    const int NXc = 2 * wc.w[0] + 1, NYc = 2 * wc.w[1] + 1;
    for (int a = 0; a < rz.n; ++a)
    for (int b = 0; b < ry.n; ++b)
    for (int c = 0; c < rx.n; ++c) {
        const int kx = rx.idx[c], ky = ry.idx[b], kz = rz.idx[a];
        const double rw = double(rx.wt[c]) * double(ry.wt[b]) * double(rz.wt[a]);
        const int64_t kp = ((int64_t)kz * df.g[1] + ky) * df.g[0] + kx;
        for (int oz = -wf.w[2]; oz <= wf.w[2]; ++oz)
        for (int oy = -wf.w[1]; oy <= wf.w[1]; ++oy)
        for (int ox = -wf.w[0]; ox <= wf.w[0]; ++ox) {
            const int o = ((oz + wf.w[2]) * NYf + (oy + wf.w[1])) * NXf + (ox + wf.w[0]);
            const c128 x = cf[o * npf + kp];
            if (x.re == 0.0 && x.im == 0.0) continue;
            const int lx = kx + ox, ly = ky + oy, lz = kz + oz;
            if (lx < 0 || lx >= df.g[0] || ly < 0 || ly >= df.g[1] || lz < 0 || lz >= df.g[2]) {
                overflow[0] = 1;                  // nonzero coupling outside the grid
                continue;
            }
            Transfer1D px, py, pz;
            px.prolong_parents(lx, nodal_mask & 1, dc.g[0]);
            py.prolong_parents(ly, nodal_mask & 2, dc.g[1]);
            if (three) pz.prolong_parents(lz, nz, dc.g[2]);
            else { pz.n = 1; pz.idx[0] = 0; pz.wt[0] = 1.0f; }
            for (int e = 0; e < pz.n; ++e)
            for (int f = 0; f < py.n; ++f)
            for (int g = 0; g < px.n; ++g) {
                // prolongation weights are 2x the restriction weights per axis
                const int dx = px.idx[g] - I, dy = py.idx[f] - J, dz = pz.idx[e] - K;
                if (dx < -wc.w[0] || dx > wc.w[0] || dy < -wc.w[1] || dy > wc.w[1] ||
                    dz < -wc.w[2] || dz > wc.w[2]) {
                    overflow[0] = 1;
                    continue;
                }
                double pw = double(px.wt[g]) * double(py.wt[f]) * double(pz.wt[e]);
                const int t = ((dz + wc.w[2]) * NYc + (dy + wc.w[1])) * NXc + (dx + wc.w[0]);
                const double s = rw * pw;
                acc[t] = acc[t] + mk(s * x.re, s * x.im);
            }
        }
    }
    for (int t = 0; t < ncs; ++t) cc[t * npc + q] = acc[t];
}

// Dense augmented matrix [A | I] (N x 2N, row-major) from a stencil.
__global__ void k_dense_from_stencil(Dims d, Widths w, const c128* __restrict__ st,
                                     c128* __restrict__ M) {
    const int64_t N = d.np();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int i = (int)(q % d.g[0]);
    const int j = (int)((q / d.g[0]) % d.g[1]);
    const int k = (int)(q / ((int64_t)d.g[0] * d.g[1]));
    c128* row = M + q * 2 * N;
    for (int64_t c = 0; c < 2 * N; ++c) row[c] = mk(0.0, 0.0);
    row[N + q] = mk(1.0, 0.0);
    const int NX = 2 * w.w[0] + 1, NY = 2 * w.w[1] + 1;
    for (int oz = -w.w[2]; oz <= w.w[2]; ++oz)
    for (int oy = -w.w[1]; oy <= w.w[1]; ++oy)
    for (int ox = -w.w[0]; ox <= w.w[0]; ++ox) {
        const int x = i + ox, y = j + oy, z = k + oz;
        if (x < 0 || x >= d.g[0] || y < 0 || y >= d.g[1] || z < 0 || z >= d.g[2]) continue;
        const int o = ((oz + w.w[2]) * NY + (oy + w.w[1])) * NX + (ox + w.w[0]);
        row[((int64_t)z * d.g[1] + y) * d.g[0] + x] = st[o * N + q];
    }
}

// Gauss-Jordan step kk, part 1: pivot = argmax_{i >= kk} |M[i][kk]| (one block).
__global__ void __launch_bounds__(256)
k_gj_pivot(int64_t N, int64_t kk, const c128* __restrict__ M, int64_t* __restrict__ piv,
           c128* __restrict__ pval) {
    __shared__ double bv[256];
    __shared__ int64_t bi[256];
    double best = -1.0;
    int64_t besti = kk;
    for (int64_t i = kk + threadIdx.x; i < N; i += blockDim.x) {
        const double a = cabs2(M[i * 2 * N + kk]);
        if (a > best) { best = a; besti = i; }
    }
    bv[threadIdx.x] = best; bi[threadIdx.x] = besti;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = bv[threadIdx.x + s];
            const int64_t oi = bi[threadIdx.x + s];
            if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = o; bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *piv = bi[0];
        *pval = M[bi[0] * 2 * N + kk];
    }
}

// part 2: swap rows kk and pivot and scale row kk by 1 / pivot value (the
// value was saved by k_gj_pivot, so no thread reads a row being rewritten).
__global__ void __launch_bounds__(256)
k_gj_swap_scale(int64_t N, int64_t kk, c128* __restrict__ M, const int64_t* __restrict__ piv,
                const c128* __restrict__ pval) {
    const int64_t pr = *piv;
    const c128 pv = *pval;
    const c128 inv = cdiv(mk(1.0, 0.0), pv);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < 2 * N;
         c += (int64_t)gridDim.x * blockDim.x) {
        const c128 a = M[kk * 2 * N + c];
        const c128 b = M[pr * 2 * N + c];
        if (pr != kk) M[pr * 2 * N + c] = a;
        M[kk * 2 * N + c] = inv * b;
    }
}

__global__ void __launch_bounds__(256)
k_gj_column(int64_t N, int64_t kk, const c128* __restrict__ M, c128* __restrict__ mult) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) mult[i] = (i == kk) ? mk(0.0, 0.0) : M[i * 2 * N + kk];
}

// part 3: M[i][c] -= mult[i] * M[kk][c] for i != kk
__global__ void __launch_bounds__(256)
k_gj_eliminate(int64_t N, int64_t kk, c128* __restrict__ M, const c128* __restrict__ mult) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (c >= 2 * N || i == kk) return;
    const c128 m = mult[i];
    if (m.re == 0.0 && m.im == 0.0) return;
    M[i * 2 * N + c] = M[i * 2 * N + c] - m * M[kk * 2 * N + c];
}

__global__ void k_gj_extract(int64_t N, const c128* __restrict__ M, c128* __restrict__ inv) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t i = t / N, c = t % N;
    inv[t] = M[i * 2 * N + N + c];
}

}  // namespace eh
