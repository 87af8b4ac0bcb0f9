// 3D coarse-level damped Jacobi sweeps, residual and first two sweeps for
// the 27-point Galerkin stencils of the mixed intergrid (eq. tildeRu1: every
// coarse operator stays 3 wide per axis), with each right-hand side's three
// planes staged in LDS (the per-sweep path of the 3D V(2,2) cycles,
// Section 4.5).
//
// A workgroup owns STX x STY points of plane k of one block's level.  Per
// right-hand side it stages planes k-1, k and k+1 of its box plus one point
// around it (u in modes 1 and 2, f in mode 5) -- coalesced along x -- into
// one of two LDS buffers and loads the next right-hand side's while this
// one is computed: one barrier per right-hand side.  The point's 27
// coefficients (in mode 5 times the neighbours' w / D) and its w / D are
// held for the whole batch.  Per point, with X u = sum_o c_o u_o summed in a
// fixed order of fused multiply-adds:
//   mode 1:  u + w D^-1 (f - X u)
//   mode 2:  f - X u
//   mode 5:  u1 = w D^-1 f;  u1 + w D^-1 (f - X u1)
// Points outside the level hold 0 and their coefficients are 0.
//
// Grid: (x tiles, y tiles, maxg2 * ns * chunks); workgroup z takes plane
// z % maxg2 of slot (z / maxg2) % ns and the chunk z / (maxg2 * ns) of rch
// right-hand sides.
#pragma once

#include "eh_common.h"
#include "eh_group_kernels.h"

namespace eh {

constexpr int STX = 32, STY = 8;

template <class T, int MODE>
__global__ void __launch_bounds__(256)
k_gstencil3_lds(GArgs<T> a, int nrhs, int rch) {
    static_assert(MODE == 1 || MODE == 2 || MODE == 5, "staged modes");
    constexpr int UW = STX + 2, UH = STY + 2, NP = UW * UH, NS = 3 * NP;
    constexpr int NR = (NS + 255) / 256;
    __shared__ cplx<T> lds[2][NS];
    const int zq = blockIdx.z / a.maxg2;
    const int k = blockIdx.z - zq * a.maxg2;
    const int slot = zq % a.ns;
    const int rlo = (zq / a.ns) * rch, rhi = min(nrhs, rlo + rch);
    const Dims d = a.d[slot];
    const int x0 = blockIdx.x * STX, y0 = blockIdx.y * STY;
    if (k >= d.g[2] || x0 >= d.g[0] || y0 >= d.g[1]) return;   // uniform per workgroup
    const int tid = threadIdx.x;
    const int tx = tid % STX, ty = tid / STX;
    const int i = x0 + tx, j = y0 + ty;
    const bool mine = i < d.g[0] && j < d.g[1];
    const int64_t sy = d.g[0], sz = (int64_t)d.g[0] * d.g[1], np = d.np();
    const int64_t p = mine ? (int64_t)k * sz + (int64_t)j * sy + i : 0;
    int64_t sidx[NR];
#pragma unroll
    for (int it = 0; it < NR; ++it) {
        const int q = tid + it * 256;
        const int pl = q / NP, e = q - pl * NP;
        const int ey = e / UW, ex = e - ey * UW;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey, gz = k - 1 + pl;
        sidx[it] = (q < NS && gx >= 0 && gx < d.g[0] && gy >= 0 && gy < d.g[1] && gz >= 0 && gz < d.g[2])
                       ? (int64_t)gz * sz + (int64_t)gy * sy + gx
                       : -1;
    }
    const cplx<T>* __restrict__ coef = a.coef[slot];
    const cplx<T>* __restrict__ dinv = a.dinv[slot];
    const cplx<T> sc = mine ? dinv[p] : czero<T>();
    cplx<T> cf[27];
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                const int o = ((oz + 1) * 3 + (oy + 1)) * 3 + (ox + 1);
                const bool ok = mine && k + oz >= 0 && k + oz < d.g[2] && j + oy >= 0 && j + oy < d.g[1] &&
                                i + ox >= 0 && i + ox < d.g[0];
                const int64_t q = p + oz * sz + oy * sy + ox;
                cf[o] = ok ? stencil_coef<T, 27, false>(coef, np, o, p, q) : czero<T>();
                if (MODE == 5) cf[o] = cf[o] * (ok ? dinv[q] : czero<T>());
            }
    const cplx<T>* __restrict__ src = MODE == 5 ? a.f[slot] : a.u[slot];
    const int64_t vsrc = MODE == 5 ? a.vf[slot] : a.vu[slot];
    const cplx<T>* __restrict__ f = a.f[slot];
    const int64_t vf = a.vf[slot];
    cplx<T>* __restrict__ out = a.out[slot];
    const int64_t vo = a.vo[slot];
    const int lc = NP + (ty + 1) * UW + (tx + 1);   // the point in the middle plane
    cplx<T> vin[NR], vff;
    auto load_in = [&](int r) {
        const cplx<T>* sr = src + (int64_t)r * vsrc;
#pragma unroll
        for (int it = 0; it < NR; ++it) vin[it] = sr[sidx[it] >= 0 ? sidx[it] : 0];
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
        const cplx<T> fr = vff;
        if (r + 1 < rhi) load_in(r + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (!mine) continue;
        cplx<T> xu = czero<T>();
#pragma unroll
        for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
            for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) {
                    const int o = ((oz + 1) * 3 + (oy + 1)) * 3 + (ox + 1);
                    xu = cfma(cf[o], S[lc + oz * NP + oy * UW + ox], xu);
                }
        cplx<T> v;
        if (MODE == 1) {
            v = cfma(sc, fr - xu, S[lc]);
        } else if (MODE == 2) {
            v = fr - xu;
        } else {
            const cplx<T> fp = S[lc];
            v = cfma(sc, fp - xu, sc * fp);
        }
        out[(int64_t)r * vo + p] = v;
    }
}

}  // namespace eh
