// 3D fine-level damped Jacobi sweeps, residual and first two sweeps with
// each right-hand side's plane staged in LDS (the per-sweep path of the
// 3D V(2,2) cycles, Section 4.4.1 and the 3D setting of Section 4.5).
//
// A workgroup owns FTX x FTY points of plane k of one block's fine grid.
// Per right-hand side it stages the plane's values of its box plus one
// point around it (u in modes 1 and 2, f in mode 5) -- every value loaded
// once, coalesced along x -- into one of two LDS buffers, reads the values
// one plane below and above straight from memory, and loads the next
// right-hand side's while this one is computed: one barrier per right-hand
// side.  The point's couplings, diagonal and first-sweep factor are held
// for the whole batch.  Arithmetic per point (fixed-order fused
// multiply-adds; the diagonal of a Jacobi update cancels algebraically):
//   mode 1:  (1 - w) u + w D^-1 (f + s(u))
//   mode 2:  f - D u + s(u)
//   mode 5:  u1 = w D^-1 f;  w D^-1 ((2 - w) f + s(u1))
// with s(v) = sum_nb c_nb v_nb over x-, x+, y-, y+, z-, z+ and, in mode 5,
// u1 of a neighbour = (w / D_nb) f_nb.  Values outside the grid are zero and
// the couplings towards them are zero.
//
// Grid: (x tiles, y tiles, maxg2 * ns * chunks); workgroup z takes plane
// z % maxg2 of slot (z / maxg2) % ns and the chunk z / (maxg2 * ns) of rch
// right-hand sides.
#pragma once

#include "eh_common.h"
#include "eh_group_kernels.h"
#include "eh_mg_kernels.h"

namespace eh {

constexpr int FTX = 32, FTY = 8;

template <class T>
__device__ __forceinline__ void fma_rc3(cplx<T>& acc, T c, cplx<T> v) {
    acc.re = fmat(c, v.re, acc.re);
    acc.im = fmat(c, v.im, acc.im);
}

template <class T, int KIND, int MODE>
__global__ void __launch_bounds__(256)
k_gfine3_lds(GArgs<T> a, int nrhs, int rch) {
    static_assert(MODE == 1 || MODE == 2 || MODE == 5, "staged modes");
    constexpr int UW = FTX + 2, UH = FTY + 2, NS = UW * UH;
    constexpr int NR = (NS + 255) / 256;
    __shared__ cplx<T> lds[2][NS];
    const int zq = blockIdx.z / a.maxg2;
    const int k = blockIdx.z - zq * a.maxg2;
    const int slot = zq % a.ns;
    const int rlo = (zq / a.ns) * rch, rhi = min(nrhs, rlo + rch);
    const Dims d = a.d[slot];
    const int x0 = blockIdx.x * FTX, y0 = blockIdx.y * FTY;
    if (k >= d.g[2] || x0 >= d.g[0] || y0 >= d.g[1]) return;   // uniform per workgroup
    const int tid = threadIdx.x;
    const int tx = tid % FTX, ty = tid / FTX;
    const int i = x0 + tx, j = y0 + ty;
    const bool mine = i < d.g[0] && j < d.g[1];
    const int64_t sy = d.g[0], sz = (int64_t)d.g[0] * d.g[1];
    const int64_t p = mine ? (int64_t)k * sz + (int64_t)j * sy + i : 0;
    int64_t sidx[NR];
#pragma unroll
    for (int it = 0; it < NR; ++it) {
        const int q = tid + it * 256;
        const int ey = q / UW, ex = q - ey * UW;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
        sidx[it] = (q < NS && gx >= 0 && gx < d.g[0] && gy >= 0 && gy < d.g[1])
                       ? (int64_t)k * sz + (int64_t)gy * sy + gx
                       : -1;
    }
    const cplx<T>* __restrict__ D = a.D[slot];
    const T damp = a.damp, omw = T(1) - damp;
    cplx<T> Dp = czero<T>(), sc = czero<T>();
    FineCoef<T, KIND, 3> c;
#pragma unroll
    for (int b = 0; b < 3; ++b) { c.cp[b] = T(0); c.cm[b] = T(0); }
    if (mine) {
        Dp = D[p];
        sc = cdiv(mk<T>(damp, T(0)), Dp);
        c.load(d, i, j, k, p, a.w[slot][0], a.w[slot][1], a.w[slot][2], a.ih[0], a.ih[1], a.ih[2]);
    }
    const bool zm = mine && k > 0, zp = mine && k + 1 < d.g[2];
    // mode 5: the couplings times the neighbours' w / D (complex)
    cplx<T> cw[6];
    if (MODE == 5) {
        const bool nb[6] = {mine && i > 0, mine && i + 1 < d.g[0], mine && j > 0, mine && j + 1 < d.g[1], zm, zp};
        const int64_t off[6] = {-1, 1, -sy, sy, -sz, sz};
        const T cc[6] = {c.cm[0], c.cp[0], c.cm[1], c.cp[1], c.cm[2], c.cp[2]};
#pragma unroll
        for (int t = 0; t < 6; ++t)
            cw[t] = nb[t] ? cc[t] * cdiv(mk<T>(damp, T(0)), D[p + off[t]]) : czero<T>();
    }
    const cplx<T>* __restrict__ src = MODE == 5 ? a.f[slot] : a.u[slot];
    const int64_t vsrc = MODE == 5 ? a.vf[slot] : a.vu[slot];
    const cplx<T>* __restrict__ f = a.f[slot];
    const int64_t vf = a.vf[slot];
    cplx<T>* __restrict__ out = a.out[slot];
    const int64_t vo = a.vo[slot];
    const int lu = (ty + 1) * UW + (tx + 1);
    cplx<T> vin[NR], vzm, vzp, vff;
    auto load_in = [&](int r) {
        const cplx<T>* sr = src + (int64_t)r * vsrc;
#pragma unroll
        for (int it = 0; it < NR; ++it) vin[it] = sr[sidx[it] >= 0 ? sidx[it] : 0];
        vzm = sr[zm ? p - sz : p];
        vzp = sr[zp ? p + sz : p];
        if (MODE != 5) vff = f[(int64_t)r * vf + p];
    };
    if (rlo < rhi) load_in(rlo);
    for (int r = rlo; r < rhi; ++r) {
        cplx<T>* S = lds[(r - rlo) & 1];
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            const int q = tid + it * 256;
            if (q < NS) S[q] = sidx[it] >= 0 ? vin[it] : czero<T>();
        }
        const cplx<T> um = zm ? vzm : czero<T>(), up = zp ? vzp : czero<T>();
        const cplx<T> fr = vff;
        if (r + 1 < rhi) load_in(r + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (!mine) continue;
        const cplx<T> uc = S[lu];
        cplx<T> v;
        if (MODE == 5) {
            cplx<T> s = mk<T>((T(2) - damp) * uc.re, (T(2) - damp) * uc.im);
            s = cfma(cw[0], S[lu - 1], s);
            s = cfma(cw[1], S[lu + 1], s);
            s = cfma(cw[2], S[lu - UW], s);
            s = cfma(cw[3], S[lu + UW], s);
            s = cfma(cw[4], um, s);
            s = cfma(cw[5], up, s);
            v = sc * s;
        } else {
            cplx<T> s = MODE == 1 ? fr : fr - Dp * uc;
            fma_rc3(s, c.cm[0], S[lu - 1]);
            fma_rc3(s, c.cp[0], S[lu + 1]);
            fma_rc3(s, c.cm[1], S[lu - UW]);
            fma_rc3(s, c.cp[1], S[lu + UW]);
            fma_rc3(s, c.cm[2], um);
            fma_rc3(s, c.cp[2], up);
            v = MODE == 1 ? cfma(sc, s, mk<T>(omw * uc.re, omw * uc.im)) : s;
        }
        out[(int64_t)r * vo + p] = v;
    }
}

}  // namespace eh
