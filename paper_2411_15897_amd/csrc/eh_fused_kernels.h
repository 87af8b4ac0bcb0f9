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
//             width smaller, and the last one writes the tile.  On the fine
//             level the coarse correction under the region is staged in LDS
//             too, and a right-hand side's loads are issued while the
//             previous one sweeps (up_body_fine).
//
// The arithmetic per point is that of the unfused kernels (k_gfine,
// k_gstencil, k_gtransfer); only the order of summation inside a stencil
// can differ.  Points outside the level's grid hold 0 in LDS, and every
// coupling towards them is 0 (the fine couplings by construction, the
// Galerkin stencils because the setup never couples outside the grid), so
// the stencil sums need no bounds tests.
//
// Launch: blockDim (threads of the tile configuration, 1D), gridDim (tiles
// x, tiles y, slots of the group x chunks of right-hand sides): workgroup
// z handles slot z % ns and right-hand sides [c * rch, min(nrhs, c * rch +
// rch)) with c = z / ns, one after the other.  Splitting a batch over
// workgroups only changes which workgroup computes a right-hand side, not
// its arithmetic.
#pragma once

#include "eh_common.h"
#include "eh_group_kernels.h"
#include "eh_mg_kernels.h"

namespace eh {

// Tile configurations (x extent, y extent, threads): the down leg's tile
// is in coarse points, the up leg's in fine points.  Large tiles amortise
// the halo on big levels; small ones give the few-thousand-point levels
// enough workgroups and keep every phase to about one round of loads per
// thread.  The autotuner picks one per level and block group.  The phase
// loops stay rolled: on small levels each compute unit runs a workgroup or
// two, so the kernel's instruction fetch from a cold cache is part of its
// latency, and unrolled code costs more there than it gains on big levels.
struct FCfg {
    int x, y, threads;
};
constexpr FCfg kFDown[] = {{32, 8, 256}, {32, 8, 512}, {16, 8, 256}, {7, 3, 128}};
constexpr FCfg kFUp[] = {{64, 16, 1024}, {64, 8, 512}, {32, 8, 256}, {16, 8, 128}};
constexpr int kFCfgs = 4;

constexpr int FUSE_MAXW = 2;
// LDS elements: down = staged u0 (support + halo) + residual of the support;
// up = u~ (tile + 2 halos) + first sweep (tile + 1 halo)
__host__ __device__ constexpr int fd_lds(int cx, int cy) {
    return (2 * cx + 2 + 2 * FUSE_MAXW) * (2 * cy + 2 + 2 * FUSE_MAXW) + (2 * cx + 2) * (2 * cy + 2);
}
__host__ __device__ constexpr int fu_lds(int tx, int ty) {
    return (tx + 4 * FUSE_MAXW) * (ty + 4 * FUSE_MAXW) + (tx + 2 * FUSE_MAXW) * (ty + 2 * FUSE_MAXW);
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumber the tiles of one slot so that every XCD gets a contiguous
// run of tiles in row-major order: neighbouring tiles, whose halos
// overlap, then read them through the same L2.  A bijection on the tiles.
__device__ __forceinline__ void xcd_tile(int& tx, int& ty) {
    const int n = gridDim.x * gridDim.y;
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    int t = b;
    if (n >= 16) {
        const int m = (n + 7) / 8;             // tiles per XCD, rounded up
        const int full = n - 8 * (m - 1);      // XCDs that get m tiles
        const int r = b % 8, q = b / 8;
        t = r < full ? r * m + q : full * m + (r - full) * (m - 1) + q;
    }
    ty = t / gridDim.x;
    tx = t - ty * gridDim.x;
}

// Barrier for the LDS phases of a leg: orders only the workgroup's LDS
// accesses.  The legs never read global memory that another thread of the
// workgroup writes in the same launch, so a right-hand side's output stores
// (and the next one's prefetched loads) need not complete at the barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// First-sweep factor w / D at point p of level l: stored on coarse levels,
// from the fine diagonal on level 0.
template <class T, bool FINE>
__device__ __forceinline__ cplx<T> fuse_sc(const GArgs<T>& a, int slot, int64_t p) {
    if (FINE) return cdiv(mk<T>(a.damp, T(0)), a.D[slot][p]);
    return a.dinv[slot][p];
}

// The operator at one point with its coefficients in registers: stored
// stencils, X u = sum_o coef_o u; fine level, X u = D u - sum_nb c_nb u_nb
// (FineCoef).  u comes from an LDS array of row pitch SX.  Every point of
// every phase goes through these same functions, so a point's value does
// not depend on which tile, or which phase of a tile, computes it.  The up
// leg keeps its own tile point's operator for both sweeps and every
// right-hand side.
//
// On the fine level the diagonal drops out of a damped Jacobi update:
// u + w D^-1 (f - D u + s) = (1 - w) u + w D^-1 (f + s), s = sum_nb c_nb u_nb,
// and, for the residual of the first sweep from zero (u = w D^-1 f at the
// point), f - X u = (1 - w) f + s.  Both are evaluated in these forms (no
// multiplication by D), with the neighbour sum as fused multiply-adds in a
// fixed order.
template <class T, bool FINE, int KIND, int WX, int WY, bool HALF = false>
struct PointOp {
    static constexpr int NST = (2 * WX + 1) * (2 * WY + 1);
    cplx<T> cf[FINE ? 1 : NST];
    FineCoef<T, KIND, 2> fc;
    cplx<T> sc;
    T omw;   // fine level: 1 - w
    __device__ __forceinline__ void load(const GArgs<T>& a, int slot, const Dims& d, int gx, int gy, int64_t p) {
        sc = fuse_sc<T, FINE>(a, slot, p);
        if (FINE) {
            fc.load(d, gx, gy, 0, p, a.w[slot][0], a.w[slot][1], a.w[slot][2], a.ih[0], a.ih[1], a.ih[2]);
            omw = T(1) - a.damp;
        } else {
            const int64_t np = d.np();
#pragma unroll
            for (int o = 0; o < (FINE ? 1 : NST); ++o) {
                const int oy = o / (2 * WX + 1) - WY, ox = o % (2 * WX + 1) - WX;
                const bool ok = !HALF || o >= NST / 2 ||
                                (gx + ox >= 0 && gx + ox < d.g[0] && gy + oy >= 0 && gy + oy < d.g[1]);
                cf[o] = ok ? stencil_coef<T, FINE ? 1 : NST, HALF>(a.coef[slot], np, o, p, p + oy * d.g[0] + ox)
                           : czero<T>();
            }
        }
    }
    // fine level: acc + sum_nb c_nb u_nb (real couplings)
    template <int SX>
    __device__ __forceinline__ cplx<T> nbsum(const cplx<T>* S, int l, cplx<T> acc) const {
        const cplx<T> e = S[l + 1], w = S[l - 1], n = S[l + SX], s = S[l - SX];
        acc.re = fmat(fc.cp[0], e.re, acc.re);
        acc.im = fmat(fc.cp[0], e.im, acc.im);
        acc.re = fmat(fc.cm[0], w.re, acc.re);
        acc.im = fmat(fc.cm[0], w.im, acc.im);
        acc.re = fmat(fc.cp[1], n.re, acc.re);
        acc.im = fmat(fc.cp[1], n.im, acc.im);
        acc.re = fmat(fc.cm[1], s.re, acc.re);
        acc.im = fmat(fc.cm[1], s.im, acc.im);
        return acc;
    }
    // stored stencils: X u with u from an LDS array of row pitch SX at local index l
    template <int SX>
    __device__ __forceinline__ cplx<T> apply(const cplx<T>* S, int l) const {
        cplx<T> xu = czero<T>();
#pragma unroll
        for (int oy = -WY; oy <= WY; ++oy)
#pragma unroll
            for (int ox = -WX; ox <= WX; ++ox)
                xu = cfma(cf[FINE ? 0 : (oy + WY) * (2 * WX + 1) + (ox + WX)], S[l + oy * SX + ox], xu);
        return xu;
    }
    // f - X u where u is the first sweep from zero (u = w D^-1 f here)
    template <int SX>
    __device__ __forceinline__ cplx<T> first_resid(const cplx<T>* S, int l, cplx<T> fp) const {
        if (FINE) return nbsum<SX>(S, l, mk<T>(omw * fp.re, omw * fp.im));
        return fp - apply<SX>(S, l);
    }
    // one damped Jacobi update u + w D^-1 (f - X u) at local index l
    template <int SX>
    __device__ __forceinline__ cplx<T> sweep(const cplx<T>* S, int l, cplx<T> fp) const {
        const cplx<T> u = S[l];
        if (FINE) return cfma(sc, nbsum<SX>(S, l, fp), mk<T>(omw * u.re, omw * u.im));
        return cfma(sc, fp - apply<SX>(S, l), u);
    }
};

// ---------------------------------------------------------------------------
// down leg: a.d = level l, a.dc = level l+1, a.f = f_l (vf), a.out = f_{l+1} (vo)

template <class T, bool FINE, int KIND, int WX, int WY, int NM, bool MIXED, int CX, int CY, int NT>
__device__ __forceinline__ void down_body(const GArgs<T>& a, int slot, cplx<T>* lds, int r0, int r1, int tile_x,
                                          int tile_y) {
    const Dims d = a.d[slot], dc = a.dc[slot];
    const int X0 = tile_x * CX, Y0 = tile_y * CY;
    if (X0 >= dc.g[0] || Y0 >= dc.g[1]) return;       // uniform per workgroup
    const int nx = d.g[0], ny = d.g[1];
    constexpr int RX = 2 * CX + 2, RY = 2 * CY + 2;   // fine support of the tile
    constexpr int UX = RX + 2 * WX, UY = RY + 2 * WY; // plus one stencil width
    const int rx0 = 2 * X0 - 1, ry0 = 2 * Y0 - 1;
    cplx<T>* U = lds;
    cplx<T>* RR = lds + UX * UY;
    using RXW = R1<(NM & 1) != 0, MIXED>;
    using RYW = R1<(NM & 2) != 0, MIXED>;
    // Small tiles with at most one support point per thread load that
    // point's operator once, before the first barrier, and keep it for
    // every right-hand side.
    constexpr bool ONE_R = RX * RY <= NT;
    const int my_ry = (int)threadIdx.x / RX, my_rx = (int)threadIdx.x - my_ry * RX;
    const int mgx = rx0 + my_rx, mgy = ry0 + my_ry;
    const bool rin = ONE_R && (int)threadIdx.x < RX * RY && mgx >= 0 && mgx < nx && mgy >= 0 && mgy < ny;
    const int64_t rp = (int64_t)mgy * nx + mgx;
    PointOp<T, FINE, KIND, WX, WY, !FINE && NM != 0 && !MIXED> rop;
    if (rin) rop.load(a, slot, d, mgx, mgy, rp);
    // The staged points of this thread (NU rounds): the point and its first-
    // sweep factor w D^-1, computed once for the whole batch.
    constexpr int NU = (UX * UY + NT - 1) / NT;
    int up_[NU];                                   // < 0: outside the grid (or the region)
    cplx<T> usc[NU];
#pragma unroll
    for (int it = 0; it < NU; ++it) {
        const int q = threadIdx.x + it * NT;
        const int uy = q / UX, ux = q - uy * UX;
        const int gx = rx0 - WX + ux, gy = ry0 - WY + uy;
        up_[it] = -1;
        usc[it] = czero<T>();
        if (q < UX * UY && gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
            up_[it] = gy * nx + gx;
            usc[it] = fuse_sc<T, FINE>(a, slot, up_[it]);
        }
    }
    // Fine level with several support points per thread: their operators
    // (four couplings and the diagonal each) are held for the whole batch.
    constexpr bool HOLD = FINE && !ONE_R;
    constexpr int NR = HOLD ? (RX * RY + NT - 1) / NT : 1;
    PointOp<T, FINE, KIND, WX, WY, false> hop[NR];
    int hp[NR], hl[NR];
    if (HOLD) {
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            const int q = threadIdx.x + it * NT;
            const int ry = q / RX, rx = q - ry * RX;
            const int gx = rx0 + rx, gy = ry0 + ry;
            hp[it] = -1;
            hl[it] = (ry + WY) * UX + (rx + WX);
            if (q < RX * RY && gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                hp[it] = gy * nx + gx;
                hop[it].load(a, slot, d, gx, gy, hp[it]);
            }
        }
    }
    // Fine level: every global load of one right-hand side (the staged
    // points and the support points' f) is issued together without branches
    // (a point outside reads element 0 and is zeroed).
    constexpr int NUF = FINE ? NU : 1, NRF = FINE ? NR : 1;
    cplx<T> inu[NUF], inr[NRF], in_fr = czero<T>();
    auto load_in = [&](int r) {
        const cplx<T>* __restrict__ f = a.f[slot] + r * a.vf[slot];
#pragma unroll
        for (int it = 0; it < NUF; ++it) inu[it] = f[up_[it] >= 0 ? up_[it] : 0];
        if (HOLD) {
#pragma unroll
            for (int it = 0; it < NRF; ++it) inr[it] = f[hp[it] >= 0 ? hp[it] : 0];
        }
        in_fr = f[rin ? rp : 0];
    };
    for (int r = r0; r < r1; ++r) {
        const cplx<T>* __restrict__ f = a.f[slot] + r * a.vf[slot];
        cplx<T> fr;
        cplx<T> fhold[NRF];
        if constexpr (FINE) {
            load_in(r);
            fr = rin ? in_fr : czero<T>();
#pragma unroll
            for (int it = 0; it < NRF; ++it) fhold[it] = inr[it];
            if (r > r0) lds_barrier();                  // LDS of the previous RHS consumed
#pragma unroll
            for (int it = 0; it < NU; ++it) {
                const int q = threadIdx.x + it * NT;
                if (q >= UX * UY) break;
                U[q] = up_[it] >= 0 ? usc[it] * inu[it] : czero<T>();
            }
            lds_barrier();
        } else {
            fr = rin ? f[rp] : czero<T>();
            if (r > r0) lds_barrier();                  // LDS of the previous RHS consumed
#pragma unroll
            for (int it = 0; it < NU; ++it) {
                const int q = threadIdx.x + it * NT;
                if (q >= UX * UY) break;
                U[q] = up_[it] >= 0 ? usc[it] * f[up_[it]] : czero<T>();
            }
            lds_barrier();
        }
        if (ONE_R) {
            if ((int)threadIdx.x < RX * RY)
                RR[threadIdx.x] =
                    rin ? rop.template first_resid<UX>(U, (my_ry + WY) * UX + (my_rx + WX), fr) : czero<T>();
        } else if (HOLD) {
#pragma unroll
            for (int it = 0; it < NR; ++it) {
                const int q = threadIdx.x + it * NT;
                if (q >= RX * RY) break;
                RR[q] = hp[it] >= 0 ? hop[it].template first_resid<UX>(U, hl[it], fhold[it]) : czero<T>();
            }
        } else {
#pragma unroll 1
            for (int it = 0; it < (RX * RY + NT - 1) / NT; ++it) {
                const int q = threadIdx.x + it * NT;
                if (q >= RX * RY) break;
                const int ry = q / RX, rx = q - ry * RX;
                const int gx = rx0 + rx, gy = ry0 + ry;
                cplx<T> v = czero<T>();
                if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                    const int64_t p = (int64_t)gy * nx + gx;
                    const int l = (ry + WY) * UX + (rx + WX);
                    PointOp<T, FINE, KIND, WX, WY, !FINE && NM != 0 && !MIXED> op;
                    op.load(a, slot, d, gx, gy, p);
                    v = op.template first_resid<UX>(U, l, f[p]);
                }
                RR[q] = v;
            }
        }
        lds_barrier();
        cplx<T>* __restrict__ out = a.out[slot] + r * a.vo[slot];
#pragma unroll 1
        for (int it = 0; it < (CX * CY + NT - 1) / NT; ++it) {
            const int q = threadIdx.x + it * NT;
            if (q >= CX * CY) break;
            const int cy = q / CX, cx = q - cy * CX;
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

template <class T, bool FINE, int CFG>
__global__ void __launch_bounds__(kFDown[CFG].threads)
k_fdown(GArgs<T> a, int nrhs, int rch) {
    constexpr int CX = kFDown[CFG].x, CY = kFDown[CFG].y, NT = kFDown[CFG].threads;
    __shared__ cplx<T> lds[fd_lds(CX, CY)];
    const int slot = blockIdx.z % a.ns;
    const int r0 = (blockIdx.z / a.ns) * rch, r1 = min(nrhs, r0 + rch);
    const int kind = a.kind[slot];           // 0: A_1, 1: A_2, 2: H_p
    int tx, ty;
    xcd_tile(tx, ty);
#define EH_FD(FI, KI, WX, WY, NM, MX) down_body<T, FI, KI, WX, WY, NM, MX, CX, CY, NT>(a, slot, lds, r0, r1, tx, ty)
    if (FINE && kind == 2 && a.tilde) {
        if (a.mixed) EH_FD(true, 2, 1, 1, 0, true);
        else EH_FD(true, 2, 1, 1, 0, false);
    } else if (FINE && a.mixed) {
        if (kind == 2) EH_FD(true, 1, 1, 1, 0, true);
        else if (kind == 0) EH_FD(true, 0, 1, 1, 1, true);
        else EH_FD(true, 0, 1, 1, 2, true);
    } else if (FINE) {
        if (kind == 2) EH_FD(true, 1, 1, 1, 0, false);
        else if (kind == 0) EH_FD(true, 0, 1, 1, 1, false);
        else EH_FD(true, 0, 1, 1, 2, false);
    } else if (a.mixed) {
        if (kind == 2) EH_FD(false, 0, 1, 1, 0, true);
        else if (kind == 0) EH_FD(false, 0, 1, 1, 1, true);
        else EH_FD(false, 0, 1, 1, 2, true);
    } else {
        if (kind == 2) EH_FD(false, 0, 2, 2, 0, false);
        else if (kind == 0) EH_FD(false, 0, 1, 2, 1, false);
        else EH_FD(false, 0, 2, 1, 2, false);
    }
#undef EH_FD
}

// ---------------------------------------------------------------------------
// up leg: a.d = level l, a.dc = level l+1, a.f = f_l (vf), a.u = e_{l+1}
// (vu), a.out = e_l (vo)

// Coarse levels (stored Galerkin stencils); the fine level has up_body_fine.
template <class T, bool FINE, int KIND, int WX, int WY, int NM, int NU2, int TX, int TY, int NT, bool HALF>
__device__ __forceinline__ void up_body(const GArgs<T>& a, int slot, cplx<T>* lds, int r0, int r1, int tile_x,
                                        int tile_y) {
    static_assert(TX * TY == NT, "one tile point per thread");
    const Dims d = a.d[slot], dc = a.dc[slot];
    const int nx = d.g[0], ny = d.g[1];
    const int tx0 = tile_x * TX, ty0 = tile_y * TY;
    if (tx0 >= nx || ty0 >= ny) return;           // uniform per workgroup
    constexpr int HX = NU2 * WX, HY = NU2 * WY;
    constexpr int AX = TX + 2 * HX, AY = TY + 2 * HY;     // u~
    constexpr int BX = TX + 2 * WX, BY = TY + 2 * WY;     // first of two sweeps
    constexpr int RING = BX * BY - TX * TY;               // its points outside the tile
    static_assert(RING <= NT, "at most one ring point per thread");
    // small operators (fine level, 3x3 stencils) of the ring point, and any
    // operator in the small-tile configuration (meant for the small levels,
    // where registers do not limit the few resident workgroups), are loaded
    // up front with the own point's, so that every global load of the kernel
    // is issued before the first barrier
    constexpr bool RING_EARLY = FINE || (2 * WX + 1) * (2 * WY + 1) <= 9 || NT <= 128;
    cplx<T>* A = lds;
    cplx<T>* B = lds + AX * AY;
    const int64_t csy = dc.g[0];
    // this thread's tile point and its operator, kept for every sweep and RHS
    const int my_y = threadIdx.x / TX, my_x = threadIdx.x - my_y * TX;
    const int mgx = tx0 + my_x, mgy = ty0 + my_y;
    const bool mine = mgx < nx && mgy < ny;
    const int64_t mp = (int64_t)mgy * nx + mgx;
    PointOp<T, FINE, KIND, WX, WY, HALF> op;
    if (mine) op.load(a, slot, d, mgx, mgy, mp);
    // this thread's ring point (first sweep only)
    int rbx = 0, rby = 0;
    {
        const int q = threadIdx.x;
        if (q < 2 * WY * BX) {                       // rows above and below the tile
            const int row = q / BX;
            rbx = q - row * BX;
            rby = row < WY ? row : TY + row;
        } else {                                     // columns left and right
            const int q2 = q - 2 * WY * BX;
            const int row = q2 / (2 * WX), cc = q2 - row * (2 * WX);
            rby = WY + row;
            rbx = cc < WX ? cc : TX + cc;
        }
    }
    const int rgx = tx0 - WX + rbx, rgy = ty0 - WY + rby;
    const bool ring = NU2 == 2 && (int)threadIdx.x < RING && rgx >= 0 && rgx < nx && rgy >= 0 && rgy < ny;
    const int64_t rp = (int64_t)rgy * nx + rgx;
    PointOp<T, FINE, KIND, WX, WY, HALF> rop;
    if (RING_EARLY && ring) rop.load(a, slot, d, rgx, rgy, rp);
    constexpr int NA = (AX * AY + NT - 1) / NT;    // at most 3 rounds
    for (int r = r0; r < r1; ++r) {
        const cplx<T>* __restrict__ f = a.f[slot] + r * a.vf[slot];
        const cplx<T>* __restrict__ ec = a.u[slot] + r * a.vu[slot];
        cplx<T>* __restrict__ out = a.out[slot] + r * a.vo[slot];
        const cplx<T> fmine = mine ? f[mp] : czero<T>();
        const cplx<T> fring = ring ? f[rp] : czero<T>();
        if (r > r0) lds_barrier();
        // u~ = w D^-1 f + P e over region A
#pragma unroll 1
        for (int it = 0; it < NA; ++it) {
            const int q = threadIdx.x + it * NT;
            if (q >= AX * AY) break;
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
        lds_barrier();
        if (NU2 == 2) {
            // first sweep on the tile (own point) and on the ring around it
            {
                const int l = (my_y + 2 * WY) * AX + (my_x + 2 * WX);
                cplx<T> v = czero<T>();
                if (mine) v = op.template sweep<AX>(A, l, fmine);
                B[(my_y + WY) * BX + my_x + WX] = v;
            }
            if ((int)threadIdx.x < RING) {
                cplx<T> v = czero<T>();
                const int l = (rby + WY) * AX + (rbx + WX);
                if (ring && RING_EARLY) {
                    v = rop.template sweep<AX>(A, l, fring);
                } else if (ring) {
                    // wide stencils: loaded here, not held across the batch
                    PointOp<T, FINE, KIND, WX, WY, HALF> wop;
                    wop.load(a, slot, d, rgx, rgy, rp);
                    v = wop.template sweep<AX>(A, l, fring);
                }
                B[rby * BX + rbx] = v;
            }
            lds_barrier();
        }
        const cplx<T>* S = NU2 == 2 ? B : A;
        constexpr int SX = NU2 == 2 ? BX : AX;
        constexpr int OX = NU2 == 2 ? WX : HX, OY = NU2 == 2 ? WY : HY;
        if (mine) {
            const int l = (my_y + OY) * SX + (my_x + OX);
            out[mp] = op.template sweep<SX>(S, l, fmine);
        }
    }
}

// Fine-level up leg.  Per right-hand side: the coarse correction e_{l+1}
// under the tile's region is staged in LDS (one load per coarse point
// instead of four per fine point), u~ = w D^-1 f + P e is formed from it,
// and the sweeps follow; the loads of the next right-hand side (its coarse
// region, f at the staged points, at the own and the ring point) are issued
// before this one's first sweep.  Two barriers per right-hand side: the
// next coarse region is written to LDS while this one sweeps (its readers,
// the staging of u~, are past the first barrier).
// LDS: coarse region, u~ region, first-sweep region.
template <int TX, int TY, int NU2>
struct FineUpGeom {
    static constexpr int HX = NU2, HY = NU2;                 // fine operators: half width 1
    static constexpr int AX = TX + 2 * HX, AY = TY + 2 * HY;
    static constexpr int BX = TX + 2, BY = TY + 2;
    static constexpr int CW = (AX + 1) / 2 + 3, CH = (AY + 1) / 2 + 3;
    static constexpr int LDS = CW * CH + AX * AY + (NU2 == 2 ? BX * BY : 0);
};

template <class T, int KIND, int NM, int NU2, int TX, int TY, int NT>
__device__ __forceinline__ void up_body_fine(const GArgs<T>& a, int slot, cplx<T>* lds, int r0, int r1, int tile_x,
                                             int tile_y) {
    static_assert(TX * TY == NT, "one tile point per thread");
    using G = FineUpGeom<TX, TY, NU2>;
    constexpr int AX = G::AX, AY = G::AY, BX = G::BX, BY = G::BY, CW = G::CW, CH = G::CH;
    constexpr int HX = G::HX, HY = G::HY;
    constexpr int RING = BX * BY - TX * TY;
    static_assert(RING <= NT, "at most one ring point per thread");
    const Dims d = a.d[slot], dc = a.dc[slot];
    const int nx = d.g[0], ny = d.g[1];
    const int tx0 = tile_x * TX, ty0 = tile_y * TY;
    if (tx0 >= nx || ty0 >= ny) return;           // uniform per workgroup
    cplx<T>* C = lds;
    cplx<T>* A = lds + CW * CH;
    cplx<T>* B = A + AX * AY;
    // coarse region: parents of every point of the u~ region
    const int cx0 = ((tx0 - HX) >> 1) - 1, cy0 = ((ty0 - HY) >> 1) - 1;
    // own tile point and its operator
    const int my_y = threadIdx.x / TX, my_x = threadIdx.x - my_y * TX;
    const int mgx = tx0 + my_x, mgy = ty0 + my_y;
    const bool mine = mgx < nx && mgy < ny;
    const int mp = mine ? mgy * nx + mgx : 0;
    PointOp<T, true, KIND, 1, 1, false> op;
    if (mine) op.load(a, slot, d, mgx, mgy, mp);
    // ring point of the first sweep (NU2 == 2)
    int rbx = 0, rby = 0;
    {
        const int q = threadIdx.x;
        if (q < 2 * BX) {
            const int row = q / BX;
            rbx = q - row * BX;
            rby = row < 1 ? row : TY + row;
        } else {
            const int q2 = q - 2 * BX;
            const int row = q2 / 2, cc = q2 - row * 2;
            rby = 1 + row;
            rbx = cc < 1 ? cc : TX + cc;
        }
    }
    const int rgx = tx0 - 1 + rbx, rgy = ty0 - 1 + rby;
    const bool ring = NU2 == 2 && (int)threadIdx.x < RING && rgx >= 0 && rgx < nx && rgy >= 0 && rgy < ny;
    const int rp = ring ? rgy * nx + rgx : 0;
    PointOp<T, true, KIND, 1, 1, false> rop;
    if (ring) rop.load(a, slot, d, rgx, rgy, rp);
    // staged points: point, first-sweep factor, parents in the LDS coarse
    // region and their weights, for the whole batch
    constexpr int NA = (AX * AY + NT - 1) / NT;
    int sp[NA], sl[NA], sdx[NA], sdy[NA];
    T sw[NA][4];
    cplx<T> ssc[NA];
#pragma unroll
    for (int it = 0; it < NA; ++it) {
        const int q = threadIdx.x + it * NT;
        const int ay = q / AX, ax = q - ay * AX;
        const int gx = tx0 - HX + ax, gy = ty0 - HY + ay;
        sp[it] = -1; sl[it] = 0; sdx[it] = 0; sdy[it] = 0;
        sw[it][0] = sw[it][1] = sw[it][2] = sw[it][3] = T(0);
        ssc[it] = czero<T>();
        if (q < AX * AY && gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
            int xi0, xi1, yi0, yi1;
            float xw0, xw1, yw0, yw1;
            p1<(NM & 1) != 0>(gx, dc.g[0], xi0, xi1, xw0, xw1);
            p1<(NM & 2) != 0>(gy, dc.g[1], yi0, yi1, yw0, yw1);
            sp[it] = gy * nx + gx;
            sl[it] = (yi0 - cy0) * CW + (xi0 - cx0);
            sdx[it] = xi1 - xi0;
            sdy[it] = (yi1 - yi0) * CW;
            sw[it][0] = T(yw0) * T(xw0);
            sw[it][1] = T(yw0) * T(xw1);
            sw[it][2] = T(yw1) * T(xw0);
            sw[it][3] = T(yw1) * T(xw1);
            ssc[it] = fuse_sc<T, true>(a, slot, sp[it]);
        }
    }
    // coarse region points of this thread
    constexpr int NC = (CW * CH + NT - 1) / NT;
    int cpt[NC];
#pragma unroll
    for (int it = 0; it < NC; ++it) {
        const int q = threadIdx.x + it * NT;
        const int cy = q / CW, cx = q - cy * CW;
        const int gx = cx0 + cx, gy = cy0 + cy;
        cpt[it] = (q < CW * CH && gx >= 0 && gx < dc.g[0] && gy >= 0 && gy < dc.g[1]) ? gy * dc.g[0] + gx : -1;
    }
    // one right-hand side's inputs, loaded without branches (a point outside
    // reads element 0 and is zeroed where it is used)
    cplx<T> vc[NC], vf[NA], vfm, vfr;
    auto load_in = [&](int r) {
        const cplx<T>* __restrict__ f = a.f[slot] + r * a.vf[slot];
        const cplx<T>* __restrict__ ec = a.u[slot] + r * a.vu[slot];
#pragma unroll
        for (int it = 0; it < NC; ++it) vc[it] = ec[cpt[it] >= 0 ? cpt[it] : 0];
#pragma unroll
        for (int it = 0; it < NA; ++it) vf[it] = f[sp[it] >= 0 ? sp[it] : 0];
        vfm = f[mp];
        vfr = f[rp];
    };
    auto store_c = [&]() {
#pragma unroll
        for (int it = 0; it < NC; ++it) {
            const int q = threadIdx.x + it * NT;
            if (q < CW * CH) C[q] = cpt[it] >= 0 ? vc[it] : czero<T>();
        }
    };
    load_in(r0);
    store_c();
    lds_barrier();
    for (int r = r0; r < r1; ++r) {
        cplx<T>* __restrict__ out = a.out[slot] + r * a.vo[slot];
        const cplx<T> fmine = mine ? vfm : czero<T>();
        const cplx<T> fring = ring ? vfr : czero<T>();
        cplx<T> fa[NA];
#pragma unroll
        for (int it = 0; it < NA; ++it) fa[it] = vf[it];
        const bool more = r + 1 < r1;
        if (more) load_in(r + 1);
        // u~ = w D^-1 f + P e over region A
#pragma unroll
        for (int it = 0; it < NA; ++it) {
            const int q = threadIdx.x + it * NT;
            if (q >= AX * AY) break;
            const cplx<T>* c0 = C + sl[it];
            const cplx<T> pe = sw[it][0] * c0[0] + sw[it][1] * c0[sdx[it]] + sw[it][2] * c0[sdy[it]] +
                               sw[it][3] * c0[sdy[it] + sdx[it]];
            A[q] = sp[it] >= 0 ? cfma(ssc[it], fa[it], pe) : czero<T>();
        }
        lds_barrier();
        if (NU2 == 2) {
            {
                const int l = (my_y + 2) * AX + (my_x + 2);
                B[(my_y + 1) * BX + my_x + 1] = mine ? op.template sweep<AX>(A, l, fmine) : czero<T>();
            }
            if ((int)threadIdx.x < RING) {
                const int l = (rby + 1) * AX + (rbx + 1);
                B[rby * BX + rbx] = ring ? rop.template sweep<AX>(A, l, fring) : czero<T>();
            }
            if (more) store_c();
            lds_barrier();
            if (mine) out[mp] = op.template sweep<BX>(B, (my_y + 1) * BX + (my_x + 1), fmine);
        } else {
            if (more) store_c();
            if (mine) out[mp] = op.template sweep<AX>(A, (my_y + 1) * AX + (my_x + 1), fmine);
            lds_barrier();
        }
    }
}

// Coarse-level up leg (stored Galerkin stencils of half widths WX, WY) on
// the same plan as the fine one: per right-hand side the coarse correction
// under the region is staged in LDS, u~ is formed from it with every
// RHS-independent quantity of a staged point (index, w D^-1, parents and
// weights) held in registers, and the next right-hand side's loads are in
// flight during the sweeps; two barriers per right-hand side.  The ring
// points' operators are staged in LDS once per workgroup when they fit
// (RING_LDS), else loaded per right-hand side.
template <class T, int WX, int WY, int NU2, int TX, int TY>
struct CoarseUpGeom {
    static constexpr int HX = NU2 * WX, HY = NU2 * WY;
    static constexpr int AX = TX + 2 * HX, AY = TY + 2 * HY;
    static constexpr int BX = TX + 2 * WX, BY = TY + 2 * WY;
    static constexpr int RING = NU2 == 2 ? BX * BY - TX * TY : 0;
    static constexpr int NST = (2 * WX + 1) * (2 * WY + 1);
    static constexpr int CW = (AX + 1) / 2 + 3, CH = (AY + 1) / 2 + 3;
    static constexpr int BASE = CW * CH + AX * AY + (NU2 == 2 ? BX * BY : 0);
    static constexpr bool RING_LDS = NU2 == 2 && (BASE + NST * RING) * (int)sizeof(cplx<T>) <= 56 * 1024;
    static constexpr int LDS = BASE + (RING_LDS ? NST * RING : 0);
};

// Interpolation weights from a code of 2 bits: 0 (1, 0), 1 (3/4, 1/4),
// 2 (1/2, 1/2), 3 (3/4, 0) -- the values p1 gives.
__device__ __forceinline__ void wcode(int c, float& w0, float& w1) {
    w0 = c == 0 ? 1.0f : (c == 2 ? 0.5f : 0.75f);
    w1 = c == 1 ? 0.25f : (c == 2 ? 0.5f : 0.0f);
}
__device__ __forceinline__ int wcode_of(float w0, float w1) {
    return w0 == 1.0f ? 0 : (w0 == 0.5f ? 2 : (w1 == 0.25f ? 1 : 3));
}

template <class T, int WX, int WY, int NM, int NU2, int TX, int TY, int NT, bool HALF>
__device__ __forceinline__ void up_body_coarse(const GArgs<T>& a, int slot, cplx<T>* lds, int r0, int r1,
                                               int tile_x, int tile_y) {
    static_assert(TX * TY == NT, "one tile point per thread");
    using G = CoarseUpGeom<T, WX, WY, NU2, TX, TY>;
    static_assert(G::LDS <= std::max(std::max(CoarseUpGeom<T, 2, 2, NU2, TX, TY>::LDS,
                                              CoarseUpGeom<T, 1, 2, NU2, TX, TY>::LDS),
                                     std::max(CoarseUpGeom<T, 2, 1, NU2, TX, TY>::LDS,
                                              CoarseUpGeom<T, 1, 1, NU2, TX, TY>::LDS)),
                  "the kernel's LDS array covers this stencil shape");
    constexpr int AX = G::AX, AY = G::AY, BX = G::BX, BY = G::BY, CW = G::CW, CH = G::CH;
    constexpr int HX = G::HX, HY = G::HY, RING = G::RING, NST = G::NST;
    constexpr bool RING_LDS = G::RING_LDS;
    static_assert(RING <= NT, "at most one ring point per thread");
    const Dims d = a.d[slot], dc = a.dc[slot];
    const int nx = d.g[0], ny = d.g[1];
    const int tx0 = tile_x * TX, ty0 = tile_y * TY;
    if (tx0 >= nx || ty0 >= ny) return;           // uniform per workgroup
    cplx<T>* C = lds;
    cplx<T>* A = C + CW * CH;
    cplx<T>* B = A + AX * AY;
    cplx<T>* RC = B + (NU2 == 2 ? BX * BY : 0);
    const int cx0 = ((tx0 - HX) >> 1) - 1, cy0 = ((ty0 - HY) >> 1) - 1;
    const int my_y = threadIdx.x / TX, my_x = threadIdx.x - my_y * TX;
    const int mgx = tx0 + my_x, mgy = ty0 + my_y;
    const bool mine = mgx < nx && mgy < ny;
    const int mp = mine ? mgy * nx + mgx : 0;
    PointOp<T, false, 0, WX, WY, HALF> op;
    if (mine) op.load(a, slot, d, mgx, mgy, mp);
    // ring point of the first sweep
    int rbx = 0, rby = 0;
    {
        const int q = threadIdx.x;
        if (q < 2 * WY * BX) {
            const int row = q / BX;
            rbx = q - row * BX;
            rby = row < WY ? row : TY + row;
        } else {
            const int q2 = q - 2 * WY * BX;
            const int row = q2 / (2 * WX), cc = q2 - row * (2 * WX);
            rby = WY + row;
            rbx = cc < WX ? cc : TX + cc;
        }
    }
    const int rgx = tx0 - WX + rbx, rgy = ty0 - WY + rby;
    const bool ring = NU2 == 2 && (int)threadIdx.x < RING && rgx >= 0 && rgx < nx && rgy >= 0 && rgy < ny;
    const int rp = ring ? rgy * nx + rgx : 0;
    cplx<T> rsc = czero<T>();
    if (RING_LDS && (int)threadIdx.x < RING) {
        const int64_t np = d.np();
#pragma unroll
        for (int o = 0; o < NST; ++o) {
            const int oy = o / (2 * WX + 1) - WY, ox = o % (2 * WX + 1) - WX;
            const bool ok = ring && (!HALF || o >= NST / 2 ||
                                     (rgx + ox >= 0 && rgx + ox < nx && rgy + oy >= 0 && rgy + oy < ny));
            RC[o * RING + threadIdx.x] = ok ? stencil_coef<T, NST, HALF>(a.coef[slot], np, o, rp, rp + oy * nx + ox)
                                            : czero<T>();
        }
        rsc = ring ? a.dinv[slot][rp] : czero<T>();
    }
    // staged points: index, w D^-1, parents in the LDS coarse region and the
    // weight codes, for the whole batch
    constexpr int NA = (AX * AY + NT - 1) / NT;
    int sp[NA], sl[NA], sk[NA];
    cplx<T> ssc[NA];
#pragma unroll
    for (int it = 0; it < NA; ++it) {
        const int q = threadIdx.x + it * NT;
        const int ay = q / AX, ax = q - ay * AX;
        const int gx = tx0 - HX + ax, gy = ty0 - HY + ay;
        sp[it] = -1; sl[it] = 0; sk[it] = 0;
        ssc[it] = czero<T>();
        if (q < AX * AY && gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
            int xi0, xi1, yi0, yi1;
            float xw0, xw1, yw0, yw1;
            p1<(NM & 1) != 0>(gx, dc.g[0], xi0, xi1, xw0, xw1);
            p1<(NM & 2) != 0>(gy, dc.g[1], yi0, yi1, yw0, yw1);
            sp[it] = gy * nx + gx;
            sl[it] = (yi0 - cy0) * CW + (xi0 - cx0);
            // bits 0-1 / 2-3: weight codes along x / y; bits 4-5 / 6-7: parent step + 1
            sk[it] = wcode_of(xw0, xw1) | (wcode_of(yw0, yw1) << 2) | ((xi1 - xi0 + 1) << 4) | ((yi1 - yi0 + 1) << 6);
            ssc[it] = a.dinv[slot][sp[it]];
        }
    }
    constexpr int NC = (CW * CH + NT - 1) / NT;
    int cpt[NC];
#pragma unroll
    for (int it = 0; it < NC; ++it) {
        const int q = threadIdx.x + it * NT;
        const int cy = q / CW, cx = q - cy * CW;
        const int gx = cx0 + cx, gy = cy0 + cy;
        cpt[it] = (q < CW * CH && gx >= 0 && gx < dc.g[0] && gy >= 0 && gy < dc.g[1]) ? gy * dc.g[0] + gx : -1;
    }
    cplx<T> vc[NC], vf[NA], vfm, vfr;
    auto load_in = [&](int r) {
        const cplx<T>* __restrict__ f = a.f[slot] + r * a.vf[slot];
        const cplx<T>* __restrict__ ec = a.u[slot] + r * a.vu[slot];
#pragma unroll
        for (int it = 0; it < NC; ++it) vc[it] = ec[cpt[it] >= 0 ? cpt[it] : 0];
#pragma unroll
        for (int it = 0; it < NA; ++it) vf[it] = f[sp[it] >= 0 ? sp[it] : 0];
        vfm = f[mp];
        vfr = f[rp];
    };
    auto store_c = [&]() {
#pragma unroll
        for (int it = 0; it < NC; ++it) {
            const int q = threadIdx.x + it * NT;
            if (q < CW * CH) C[q] = cpt[it] >= 0 ? vc[it] : czero<T>();
        }
    };
    load_in(r0);
    store_c();
    lds_barrier();
    for (int r = r0; r < r1; ++r) {
        cplx<T>* __restrict__ out = a.out[slot] + r * a.vo[slot];
        const cplx<T> fmine = mine ? vfm : czero<T>();
        const cplx<T> fring = ring ? vfr : czero<T>();
        cplx<T> fa[NA];
#pragma unroll
        for (int it = 0; it < NA; ++it) fa[it] = vf[it];
        const bool more = r + 1 < r1;
        if (more) load_in(r + 1);
#pragma unroll
        for (int it = 0; it < NA; ++it) {
            const int q = threadIdx.x + it * NT;
            if (q >= AX * AY) break;
            float xw0, xw1, yw0, yw1;
            wcode(sk[it] & 3, xw0, xw1);
            wcode((sk[it] >> 2) & 3, yw0, yw1);
            const int dx = ((sk[it] >> 4) & 3) - 1, dy = (((sk[it] >> 6) & 3) - 1) * CW;
            const cplx<T>* c0 = C + sl[it];
            const cplx<T> pe = (T(yw0) * T(xw0)) * c0[0] + (T(yw0) * T(xw1)) * c0[dx] + (T(yw1) * T(xw0)) * c0[dy] +
                               (T(yw1) * T(xw1)) * c0[dy + dx];
            A[q] = sp[it] >= 0 ? cfma(ssc[it], fa[it], pe) : czero<T>();
        }
        lds_barrier();
        if (NU2 == 2) {
            B[(my_y + WY) * BX + my_x + WX] =
                mine ? op.template sweep<AX>(A, (my_y + 2 * WY) * AX + (my_x + 2 * WX), fmine) : czero<T>();
            if ((int)threadIdx.x < RING) {
                const int l = (rby + WY) * AX + (rbx + WX);
                cplx<T> v = czero<T>();
                if (ring && RING_LDS) {
                    // the same PointOp code as every other point, fed from LDS
                    PointOp<T, false, 0, WX, WY, HALF> wop;
#pragma unroll
                    for (int o = 0; o < NST; ++o) wop.cf[o] = RC[o * RING + threadIdx.x];
                    wop.sc = rsc;
                    v = wop.template sweep<AX>(A, l, fring);
                } else if (ring) {
                    PointOp<T, false, 0, WX, WY, HALF> wop;
                    wop.load(a, slot, d, rgx, rgy, rp);
                    v = wop.template sweep<AX>(A, l, fring);
                }
                B[rby * BX + rbx] = v;
            }
            if (more) store_c();
            lds_barrier();
            if (mine) out[mp] = op.template sweep<BX>(B, (my_y + WY) * BX + (my_x + WX), fmine);
        } else {
            if (more) store_c();
            if (mine) out[mp] = op.template sweep<AX>(A, (my_y + HY) * AX + (my_x + HX), fmine);
            lds_barrier();
        }
    }
}

template <class T, bool FINE, int NU2, int CFG>
__global__ void __launch_bounds__(kFUp[CFG].threads)
k_fup(GArgs<T> a, int nrhs, int rch) {
    constexpr int TX = kFUp[CFG].x, TY = kFUp[CFG].y, NT = kFUp[CFG].threads;
    // every stencil shape the coarse levels use: 5x5, 3x5, 5x3, 3x3
    constexpr int LDS_N = FINE ? FineUpGeom<TX, TY, NU2>::LDS
                               : std::max(std::max(CoarseUpGeom<T, 2, 2, NU2, TX, TY>::LDS,
                                                   CoarseUpGeom<T, 1, 2, NU2, TX, TY>::LDS),
                                          std::max(CoarseUpGeom<T, 2, 1, NU2, TX, TY>::LDS,
                                                   CoarseUpGeom<T, 1, 1, NU2, TX, TY>::LDS));
    __shared__ cplx<T> lds[LDS_N];
    const int slot = blockIdx.z % a.ns;
    const int r0 = (blockIdx.z / a.ns) * rch, r1 = min(nrhs, r0 + rch);
    const int kind = a.kind[slot];
    int tx, ty;
    xcd_tile(tx, ty);
#define EH_FU(FI, KI, WX, WY, NM, HF) \
    up_body<T, FI, KI, WX, WY, NM, NU2, TX, TY, NT, HF>(a, slot, lds, r0, r1, tx, ty)
#define EH_FUF(KI, NM) up_body_fine<T, KI, NM, NU2, TX, TY, NT>(a, slot, lds, r0, r1, tx, ty)
#define EH_FUC(WX, WY, NM, HF) up_body_coarse<T, WX, WY, NM, NU2, TX, TY, NT, HF>(a, slot, lds, r0, r1, tx, ty)
    if (FINE) {
        if (kind == 2 && a.tilde) EH_FUF(2, 0);
        else if (kind == 2) EH_FUF(1, 0);
        else if (kind == 0) EH_FUF(0, 1);
        else EH_FUF(0, 2);
    } else if (a.mixed) {
        if (kind == 2) EH_FUC(1, 1, 0, false);
        else if (kind == 0) EH_FUC(1, 1, 1, false);
        else EH_FUC(1, 1, 2, false);
    } else {
        // full weighting: the shear blocks' stencils are stored half
        if (kind == 2) EH_FUC(2, 2, 0, false);
        else if (kind == 0) EH_FUC(1, 2, 1, true);
        else EH_FUC(2, 1, 2, true);
    }
#undef EH_FUC
#undef EH_FUF
#undef EH_FU
}

}  // namespace eh
