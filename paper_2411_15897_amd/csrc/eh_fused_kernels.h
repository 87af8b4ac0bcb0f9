// Fused multigrid legs for 2D V(1, nu2) cycles (nu2 = 1 or 2) started from
// a zero guess -- the cycle the preconditioner applies to every acoustic
// block (Section 4.4.1; V-cycle, one pre- and two post-smoothing damped
// Jacobi sweeps in 2D).
//
// With a zero initial guess the pre-smoothing sweep is pointwise,
// u0 = w D^-1 f, so one level's work splits into two launches:
//
//   down leg  f_{l+1} = R (f_l - X_l u0)
//             Each workgroup owns a tile of coarse points.  u0 over the
//             tile's fine support plus one stencil width is staged in LDS,
//             the residual of the support is formed from LDS into a second
//             LDS array, and every coarse point sums its restriction
//             weights (eqs. Ru1, Rp; eq. tildeRu1 for the mixed variant).
//             u0 itself is never stored.
//   up leg    e_l = S^nu2 (u0 + P e_{l+1})
//             Each workgroup owns a tile of fine points.  u~ = u0 + P e over
//             the tile plus nu2 stencil widths is staged in LDS; each
//             damped Jacobi sweep runs from LDS on a region one stencil
//             width smaller, and the last one writes the tile.
//
// The arithmetic per point is that of the unfused kernels (k_gfine,
// k_gstencil, k_gtransfer); only the order of summation inside a stencil
// can differ.  Points outside the level's grid hold 0 in LDS, and every
// coupling towards them is 0 (the fine couplings by construction, the
// Galerkin stencils because the setup never couples outside the grid), so
// the stencil sums need no bounds tests.
//
// Launch: blockDim 256 (1D), gridDim (tiles x, tiles y, slots of the group).
#pragma once

#include "eh_common.h"
#include "eh_group_kernels.h"
#include "eh_mg_kernels.h"

namespace eh {

constexpr int FUSE_THREADS = 256;
// down leg: coarse tile; up leg: fine tile
constexpr int FD_CX = 32, FD_CY = 8;
constexpr int FU_TX = 64, FU_TY = 8;
constexpr int FUSE_MAXW = 2;
// LDS elements: down = staged u0 (support + halo) + residual of the support;
// up = u~ (tile + 2 halos) + first sweep (tile + 1 halo)
constexpr int FD_LDS = (2 * FD_CX + 2 + 2 * FUSE_MAXW) * (2 * FD_CY + 2 + 2 * FUSE_MAXW) +
                       (2 * FD_CX + 2) * (2 * FD_CY + 2);
constexpr int FU_LDS = (FU_TX + 4 * FUSE_MAXW) * (FU_TY + 4 * FUSE_MAXW) +
                       (FU_TX + 2 * FUSE_MAXW) * (FU_TY + 2 * FUSE_MAXW);

// First-sweep factor w / D at point p of level l: stored on coarse levels,
// from the fine diagonal on level 0.
template <class T, bool FINE>
__device__ __forceinline__ cplx<T> fuse_sc(const GArgs<T>& a, int slot, int64_t p) {
    if (FINE) return cdiv(mk<T>(a.damp, T(0)), a.D[slot][p]);
    return a.dinv[slot][p];
}

// X u at point (gx, gy) (linear index p) with u taken from an LDS array S
// of row pitch SX at local index l.  Stored stencils: X u = sum_o coef_o u;
// fine level: X u = D u - sum_nb c_nb u_nb (FineCoef).
template <class T, bool FINE, int KIND, int WX, int WY, int SX>
__device__ __forceinline__ cplx<T> fuse_apply(const GArgs<T>& a, int slot, const Dims& d, int gx, int gy,
                                              int64_t p, const cplx<T>* S, int l) {
    if (FINE) {
        FineCoef<T, KIND, 2> c;
        c.load(d, gx, gy, 0, p, a.w[slot][0], a.w[slot][1], a.w[slot][2], a.ih[0], a.ih[1], a.ih[2]);
        const cplx<T> offs = c.cp[0] * S[l + 1] + c.cm[0] * S[l - 1] + c.cp[1] * S[l + SX] + c.cm[1] * S[l - SX];
        return a.D[slot][p] * S[l] - offs;
    }
    const int64_t np = d.np();
    const cplx<T>* __restrict__ coef = a.coef[slot];
    cplx<T> xu = czero<T>();
#pragma unroll
    for (int oy = -WY; oy <= WY; ++oy)
#pragma unroll
        for (int ox = -WX; ox <= WX; ++ox) {
            const int o = (oy + WY) * (2 * WX + 1) + (ox + WX);
            xu = xu + coef[o * np + p] * S[l + oy * SX + ox];
        }
    return xu;
}

// ---------------------------------------------------------------------------
// down leg: a.d = level l, a.dc = level l+1, a.f = f_l (vf), a.out = f_{l+1} (vo)

template <class T, bool FINE, int KIND, int WX, int WY, int NM, bool MIXED>
__device__ __forceinline__ void down_body(const GArgs<T>& a, int slot, cplx<T>* lds, int nrhs) {
    const Dims d = a.d[slot], dc = a.dc[slot];
    const int X0 = blockIdx.x * FD_CX, Y0 = blockIdx.y * FD_CY;
    if (X0 >= dc.g[0] || Y0 >= dc.g[1]) return;       // uniform per workgroup
    const int nx = d.g[0], ny = d.g[1];
    constexpr int RX = 2 * FD_CX + 2, RY = 2 * FD_CY + 2;   // fine support of the tile
    constexpr int UX = RX + 2 * WX, UY = RY + 2 * WY;       // plus one stencil width
    const int rx0 = 2 * X0 - 1, ry0 = 2 * Y0 - 1;
    cplx<T>* U = lds;
    cplx<T>* RR = lds + UX * UY;
    using RXW = R1<(NM & 1) != 0, MIXED>;
    using RYW = R1<(NM & 2) != 0, MIXED>;
    for (int r = 0; r < nrhs; ++r) {
        const cplx<T>* __restrict__ f = a.f[slot] + r * a.vf[slot];
        if (r > 0) __syncthreads();                 // LDS of the previous RHS consumed
        for (int q = threadIdx.x; q < UX * UY; q += FUSE_THREADS) {
            const int uy = q / UX, ux = q - uy * UX;
            const int gx = rx0 - WX + ux, gy = ry0 - WY + uy;
            cplx<T> v = czero<T>();
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const int64_t p = (int64_t)gy * nx + gx;
                v = fuse_sc<T, FINE>(a, slot, p) * f[p];
            }
            U[q] = v;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < RX * RY; q += FUSE_THREADS) {
            const int ry = q / RX, rx = q - ry * RX;
            const int gx = rx0 + rx, gy = ry0 + ry;
            cplx<T> v = czero<T>();
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const int64_t p = (int64_t)gy * nx + gx;
                const int l = (ry + WY) * UX + (rx + WX);
                v = f[p] - fuse_apply<T, FINE, KIND, WX, WY, UX>(a, slot, d, gx, gy, p, U, l);
            }
            RR[q] = v;
        }
        __syncthreads();
        cplx<T>* __restrict__ out = a.out[slot] + r * a.vo[slot];
        for (int q = threadIdx.x; q < FD_CX * FD_CY; q += FUSE_THREADS) {
            const int cy = q / FD_CX, cx = q - cy * FD_CX;
            const int I = X0 + cx, J = Y0 + cy;
            if (I >= dc.g[0] || J >= dc.g[1]) continue;
            // first fine index of the support, local to the region
            const int lx = 2 * cx + RXW::FIRST + 1, ly = 2 * cy + RYW::FIRST + 1;
            cplx<T> s = czero<T>();
#pragma unroll
            for (int b = 0; b < RYW::S; ++b) {
                const T wy = T(RYW::w(b));
#pragma unroll
                for (int t = 0; t < RXW::S; ++t) s = s + (wy * T(RXW::w(t))) * RR[(ly + b) * RX + lx + t];
            }
            out[(int64_t)J * dc.g[0] + I] = s;
        }
    }
}

template <class T, bool FINE>
__global__ void __launch_bounds__(FUSE_THREADS)
k_fdown(GArgs<T> a, int nrhs) {
    __shared__ cplx<T> lds[FD_LDS];
    const int slot = blockIdx.z;
    if (slot >= a.ns) return;
    const int kind = a.kind[slot];           // 0: A_1, 1: A_2, 2: H_p
    if (FINE && a.mixed) {
        if (kind == 2) down_body<T, true, 1, 1, 1, 0, true>(a, slot, lds, nrhs);
        else if (kind == 0) down_body<T, true, 0, 1, 1, 1, true>(a, slot, lds, nrhs);
        else down_body<T, true, 0, 1, 1, 2, true>(a, slot, lds, nrhs);
    } else if (FINE) {
        if (kind == 2) down_body<T, true, 1, 1, 1, 0, false>(a, slot, lds, nrhs);
        else if (kind == 0) down_body<T, true, 0, 1, 1, 1, false>(a, slot, lds, nrhs);
        else down_body<T, true, 0, 1, 1, 2, false>(a, slot, lds, nrhs);
    } else if (a.mixed) {
        if (kind == 2) down_body<T, false, 0, 1, 1, 0, true>(a, slot, lds, nrhs);
        else if (kind == 0) down_body<T, false, 0, 1, 1, 1, true>(a, slot, lds, nrhs);
        else down_body<T, false, 0, 1, 1, 2, true>(a, slot, lds, nrhs);
    } else {
        if (kind == 2) down_body<T, false, 0, 2, 2, 0, false>(a, slot, lds, nrhs);
        else if (kind == 0) down_body<T, false, 0, 1, 2, 1, false>(a, slot, lds, nrhs);
        else down_body<T, false, 0, 2, 1, 2, false>(a, slot, lds, nrhs);
    }
}

// ---------------------------------------------------------------------------
// up leg: a.d = level l, a.dc = level l+1, a.f = f_l (vf), a.u = e_{l+1}
// (vu), a.out = e_l (vo)

template <class T, bool FINE, int KIND, int WX, int WY, int NM, int NU2>
__device__ __forceinline__ void up_body(const GArgs<T>& a, int slot, cplx<T>* lds, int nrhs) {
    const Dims d = a.d[slot], dc = a.dc[slot];
    const int nx = d.g[0], ny = d.g[1];
    const int tx0 = blockIdx.x * FU_TX, ty0 = blockIdx.y * FU_TY;
    if (tx0 >= nx || ty0 >= ny) return;           // uniform per workgroup
    constexpr int HX = NU2 * WX, HY = NU2 * WY;
    constexpr int AX = FU_TX + 2 * HX, AY = FU_TY + 2 * HY;     // u~
    constexpr int BX = FU_TX + 2 * WX, BY = FU_TY + 2 * WY;     // first of two sweeps
    cplx<T>* A = lds;
    cplx<T>* B = lds + AX * AY;
    const int64_t csy = dc.g[0];
    for (int r = 0; r < nrhs; ++r) {
        const cplx<T>* __restrict__ f = a.f[slot] + r * a.vf[slot];
        const cplx<T>* __restrict__ ec = a.u[slot] + r * a.vu[slot];
        cplx<T>* __restrict__ out = a.out[slot] + r * a.vo[slot];
        if (r > 0) __syncthreads();
        for (int q = threadIdx.x; q < AX * AY; q += FUSE_THREADS) {
            const int ay = q / AX, ax = q - ay * AX;
            const int gx = tx0 - HX + ax, gy = ty0 - HY + ay;
            cplx<T> v = czero<T>();
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const int64_t p = (int64_t)gy * nx + gx;
                int xi0, xi1, yi0, yi1;
                float xw0, xw1, yw0, yw1;
                p1<(NM & 1) != 0>(gx, dc.g[0], xi0, xi1, xw0, xw1);
                p1<(NM & 2) != 0>(gy, dc.g[1], yi0, yi1, yw0, yw1);
                const cplx<T> pe = (T(yw0) * T(xw0)) * ec[yi0 * csy + xi0] +
                                   (T(yw0) * T(xw1)) * ec[yi0 * csy + xi1] +
                                   (T(yw1) * T(xw0)) * ec[yi1 * csy + xi0] +
                                   (T(yw1) * T(xw1)) * ec[yi1 * csy + xi1];
                v = fuse_sc<T, FINE>(a, slot, p) * f[p] + pe;
            }
            A[q] = v;
        }
        __syncthreads();
        if (NU2 == 2) {
            for (int q = threadIdx.x; q < BX * BY; q += FUSE_THREADS) {
                const int by = q / BX, bx = q - by * BX;
                const int gx = tx0 - WX + bx, gy = ty0 - WY + by;
                cplx<T> v = czero<T>();
                if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                    const int64_t p = (int64_t)gy * nx + gx;
                    const int l = (by + WY) * AX + (bx + WX);
                    const cplx<T> xu = fuse_apply<T, FINE, KIND, WX, WY, AX>(a, slot, d, gx, gy, p, A, l);
                    v = A[l] + fuse_sc<T, FINE>(a, slot, p) * (f[p] - xu);
                }
                B[q] = v;
            }
            __syncthreads();
        }
        const cplx<T>* S = NU2 == 2 ? B : A;
        constexpr int SX = NU2 == 2 ? BX : AX;
        for (int q = threadIdx.x; q < FU_TX * FU_TY; q += FUSE_THREADS) {
            const int ty = q / FU_TX, tx = q - ty * FU_TX;
            const int gx = tx0 + tx, gy = ty0 + ty;
            if (gx >= nx || gy >= ny) continue;
            const int64_t p = (int64_t)gy * nx + gx;
            const int l = (ty + WY) * SX + (tx + WX);
            const cplx<T> xu = fuse_apply<T, FINE, KIND, WX, WY, SX>(a, slot, d, gx, gy, p, S, l);
            out[p] = S[l] + fuse_sc<T, FINE>(a, slot, p) * (f[p] - xu);
        }
    }
}

template <class T, bool FINE, int NU2>
__global__ void __launch_bounds__(FUSE_THREADS)
k_fup(GArgs<T> a, int nrhs) {
    __shared__ cplx<T> lds[FU_LDS];
    const int slot = blockIdx.z;
    if (slot >= a.ns) return;
    const int kind = a.kind[slot];
    if (FINE) {
        if (kind == 2) up_body<T, true, 1, 1, 1, 0, NU2>(a, slot, lds, nrhs);
        else if (kind == 0) up_body<T, true, 0, 1, 1, 1, NU2>(a, slot, lds, nrhs);
        else up_body<T, true, 0, 1, 1, 2, NU2>(a, slot, lds, nrhs);
    } else if (a.mixed) {
        if (kind == 2) up_body<T, false, 0, 1, 1, 0, NU2>(a, slot, lds, nrhs);
        else if (kind == 0) up_body<T, false, 0, 1, 1, 1, NU2>(a, slot, lds, nrhs);
        else up_body<T, false, 0, 1, 1, 2, NU2>(a, slot, lds, nrhs);
    } else {
        if (kind == 2) up_body<T, false, 0, 2, 2, 0, NU2>(a, slot, lds, nrhs);
        else if (kind == 0) up_body<T, false, 0, 1, 2, 1, NU2>(a, slot, lds, nrhs);
        else up_body<T, false, 0, 2, 1, 2, NU2>(a, slot, lds, nrhs);
    }
}

}  // namespace eh
