// 3D fine-level damped Jacobi sweeps, residual and first two sweeps with
// each right-hand side's planes staged in LDS (the per-sweep path of the
// 3D V(2,2) cycles, Section 4.4.1 and the 3D setting of Section 4.5).
//
// A workgroup owns FTX x FTY points of planes k0 = 2 kb and k0 + 1 of one
// block's fine grid.  Per right-hand side it stages both planes' values of
// its box plus one point around it (u in modes 1 and 2, f in mode 5) --
// every value loaded once, coalesced along x -- into one of two LDS
// buffers, so each plane takes one z neighbour from LDS (k0 the plane
// above, k0 + 1 the plane below) and the other (k0 - 1, k0 + 2) straight
// from memory; the next right-hand side's values are loaded while this one
// is computed: one barrier per right-hand side.  The points' couplings,
// diagonals and first-sweep factors are held for the whole batch; in mode
// 5 the neighbours' w / D come from both planes' boxes, computed once per
// launch into LDS.
// Arithmetic per point (fixed-order fused multiply-adds; the diagonal of a
// Jacobi update cancels algebraically):
//   mode 1:  (1 - w) u + w D^-1 (f + s(u))
//   mode 2:  f - D u + s(u)
//   mode 5:  u1 = w D^-1 f;  w D^-1 ((2 - w) f + s(u1))
// with s(v) = sum_nb c_nb v_nb over x-, x+, y-, y+, z-, z+ and, in mode 5,
// u1 of a neighbour = (w / D_nb) f_nb.  Values outside the grid are zero and
// the couplings towards them are zero; with an odd number of planes the
// last workgroup of a column has one plane.
//
// Grid: (x tiles, y tiles, ceil(maxg2 / 2) * ns * chunks); workgroup z
// takes the plane pair z % ceil(maxg2 / 2) of slot (z / ceil(maxg2 / 2)) %
// ns and the chunk z / (ceil(maxg2 / 2) * ns) of rch right-hand sides.
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
    __shared__ cplx<T> lds[2][2][NS];
    const int nzb = (a.maxg2 + 1) / 2;
    const int zq = blockIdx.z / nzb;
    const int k0 = 2 * (blockIdx.z - zq * nzb);
    const int slot = zq % a.ns;
    const int rlo = (zq / a.ns) * rch, rhi = min(nrhs, rlo + rch);
    const Dims d = a.d[slot];
    const int x0 = blockIdx.x * FTX, y0 = blockIdx.y * FTY;
    if (k0 >= d.g[2] || x0 >= d.g[0] || y0 >= d.g[1]) return;   // uniform per workgroup
    const int tid = threadIdx.x;
    const int tx = tid % FTX, ty = tid / FTX;
    const int i = x0 + tx, j = y0 + ty;
    const bool pl1 = k0 + 1 < d.g[2];            // the second plane exists
    const bool inxy = i < d.g[0] && j < d.g[1];
    const bool mine[2] = {inxy, inxy && pl1};
    const int64_t sy = d.g[0], sz = (int64_t)d.g[0] * d.g[1];
    int64_t p[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) p[h] = mine[h] ? (int64_t)(k0 + h) * sz + (int64_t)j * sy + i : 0;
    int64_t sxy[NR];
#pragma unroll
    for (int it = 0; it < NR; ++it) {
        const int q = tid + it * 256;
        const int ey = q / UW, ex = q - ey * UW;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
        sxy[it] = (q < NS && gx >= 0 && gx < d.g[0] && gy >= 0 && gy < d.g[1]) ? (int64_t)gy * sy + gx : -1;
    }
    const int lu = (ty + 1) * UW + (tx + 1);    // the point in its plane's box
    const cplx<T>* __restrict__ D = a.D[slot];
    const T damp = a.damp, omw = T(1) - damp;
    // mode 5: w / D over both planes' boxes, once per launch, for the
    // neighbours' first-sweep factors
    __shared__ cplx<T> wd[2][MODE == 5 ? NS : 1];
    if (MODE == 5) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int it = 0; it < NR; ++it) {
                const int q = tid + it * 256;
                if (q < NS)
                    wd[h][q] = (sxy[it] >= 0 && (h == 0 || pl1))
                                   ? cdiv(mk<T>(damp, T(0)), D[(int64_t)(k0 + h) * sz + sxy[it]])
                                   : czero<T>();
            }
        __syncthreads();
    }
    cplx<T> Dp[2], sc[2];
    FineCoef<T, KIND, 3> c[2];
    cplx<T> cw[2][6];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        Dp[h] = czero<T>();
        sc[h] = czero<T>();
#pragma unroll
        for (int b = 0; b < 3; ++b) { c[h].cp[b] = T(0); c[h].cm[b] = T(0); }
        if (mine[h]) {
            Dp[h] = D[p[h]];
            sc[h] = cdiv(mk<T>(damp, T(0)), Dp[h]);
            c[h].load(d, i, j, k0 + h, p[h], a.w[slot][0], a.w[slot][1], a.w[slot][2], a.ih[0], a.ih[1], a.ih[2]);
        }
        if (MODE == 5) {
            const int k = k0 + h;
            const bool nb[6] = {mine[h] && i > 0, mine[h] && i + 1 < d.g[0], mine[h] && j > 0,
                                mine[h] && j + 1 < d.g[1], mine[h] && k > 0, mine[h] && k + 1 < d.g[2]};
            const T cc[6] = {c[h].cm[0], c[h].cp[0], c[h].cm[1], c[h].cp[1], c[h].cm[2], c[h].cp[2]};
            // w / D of the six neighbours: the own plane's box, the other
            // plane's point, and the outer plane from memory
            const bool outer = h == 0 ? nb[4] : nb[5];
            const cplx<T> wo = outer ? cdiv(mk<T>(damp, T(0)), D[h == 0 ? p[0] - sz : p[1] + sz]) : czero<T>();
            const cplx<T> wn[6] = {wd[h][lu - 1], wd[h][lu + 1], wd[h][lu - UW], wd[h][lu + UW],
                                   h == 0 ? wo : wd[0][lu], h == 0 ? wd[1][lu] : wo};
#pragma unroll
            for (int t = 0; t < 6; ++t) cw[h][t] = nb[t] ? cc[t] * wn[t] : czero<T>();
        }
    }
    const bool zm0 = mine[0] && k0 > 0, zp1 = mine[1] && k0 + 2 < d.g[2];
    const cplx<T>* __restrict__ src = MODE == 5 ? a.f[slot] : a.u[slot];
    const int64_t vsrc = MODE == 5 ? a.vf[slot] : a.vu[slot];
    const cplx<T>* __restrict__ f = a.f[slot];
    const int64_t vf = a.vf[slot];
    cplx<T>* __restrict__ out = a.out[slot];
    const int64_t vo = a.vo[slot];
    cplx<T> vin[2][NR], vzm, vzp, vff[2];
    auto load_in = [&](int r) {
        const cplx<T>* sr = src + (int64_t)r * vsrc;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int it = 0; it < NR; ++it)
                vin[h][it] = sr[(sxy[it] >= 0 && (h == 0 || pl1)) ? (int64_t)(k0 + h) * sz + sxy[it] : 0];
        vzm = sr[zm0 ? p[0] - sz : 0];
        vzp = sr[zp1 ? p[1] + sz : 0];
        if (MODE != 5) {
#pragma unroll
            for (int h = 0; h < 2; ++h) vff[h] = f[(int64_t)r * vf + p[h]];
        }
    };
    if (rlo < rhi) load_in(rlo);
    for (int r = rlo; r < rhi; ++r) {
        cplx<T>* S0 = lds[(r - rlo) & 1][0];
        cplx<T>* S1 = lds[(r - rlo) & 1][1];
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            const int q = tid + it * 256;
            if (q < NS) {
                S0[q] = sxy[it] >= 0 ? vin[0][it] : czero<T>();
                S1[q] = (sxy[it] >= 0 && pl1) ? vin[1][it] : czero<T>();
            }
        }
        const cplx<T> um0 = zm0 ? vzm : czero<T>(), up1 = zp1 ? vzp : czero<T>();
        const cplx<T> fr[2] = {vff[0], vff[1]};
        if (r + 1 < rhi) load_in(r + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!mine[h]) continue;
            const cplx<T>* S = h == 0 ? S0 : S1;
            const cplx<T> uc = S[lu];
            const cplx<T> um = h == 0 ? um0 : S0[lu];
            const cplx<T> up = h == 0 ? S1[lu] : up1;
            cplx<T> v;
            if (MODE == 5) {
                cplx<T> s = mk<T>((T(2) - damp) * uc.re, (T(2) - damp) * uc.im);
                s = cfma(cw[h][0], S[lu - 1], s);
                s = cfma(cw[h][1], S[lu + 1], s);
                s = cfma(cw[h][2], S[lu - UW], s);
                s = cfma(cw[h][3], S[lu + UW], s);
                s = cfma(cw[h][4], um, s);
                s = cfma(cw[h][5], up, s);
                v = sc[h] * s;
            } else {
                cplx<T> s = MODE == 1 ? fr[h] : fr[h] - Dp[h] * uc;
                fma_rc3(s, c[h].cm[0], S[lu - 1]);
                fma_rc3(s, c[h].cp[0], S[lu + 1]);
                fma_rc3(s, c[h].cm[1], S[lu - UW]);
                fma_rc3(s, c[h].cp[1], S[lu + UW]);
                fma_rc3(s, c[h].cm[2], um);
                fma_rc3(s, c[h].cp[2], up);
                v = MODE == 1 ? cfma(sc[h], s, mk<T>(omw * uc.re, omw * uc.im)) : s;
            }
            out[(int64_t)r * vo + p[h]] = v;
        }
    }
}

}  // namespace eh
