// Elastic operator, distributor and coupling kernels (FP64 inputs).
//
//  k_op2_lds / k_op3_lds: y = H x (eq. mixed-discretized), every field in
//      one launch (2D / 3D).
//  k_distribute: t = B r_u - A_p r_p (eq. mixed-distributed) with
//      A_p r = B B^T (mu r) - w^2 rho (1 - i gamma/w) r (eq. Ap), written in
//      the multigrid precision.  With rs given, the input of RHS r is
//      rs[r * rss] times the stored vector (an unnormalised Krylov column).
//
// Same launch shape as the multigrid kernels.
#pragma once

#include "eh_common.h"
#include "eh_mg_kernels.h"

namespace eh {

// Residual form (RES), for the FGMRES cycle starts: the launch writes
// r = b - H x instead of H x and, per right-hand side, one partial sum of
// |r|^2 per workgroup (a butterfly within each wavefront, then the four
// wavefronts, in a fixed order), which k_reduce_partials adds up -- the
// subtraction and the norm pass need not read the vectors again.
// blockDim 256; every thread takes part in the sums, points outside the
// field with zeros.
struct ResArgs {
    const c128* b;       // right-hand sides, same layout and stride as y
    c128* partial;       // [rhs][workgroup]
    int nblk;            // workgroups over all launches of one application
    int blk0;            // first workgroup index of this launch
};

__device__ __forceinline__ void res_partial(const ResArgs& ra, int r, int kz, double v) {
    __shared__ double sv[4];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) sv[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        // the workgroup's place in the plane grid (kz = its plane), not its
        // chunk of the batch: every chunk writes the rows of its own RHS
        const int blk = ra.blk0 + (kz * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        ra.partial[(int64_t)r * ra.nblk + blk] = mk((sv[0] + sv[1]) + (sv[2] + sv[3]), 0.0);
    }
    __syncthreads();       // sv is reused by the next right-hand side
}

// Operator coefficients of one launch: per face field a the couplings of
// A_a along each axis and its complex diagonal, C = 1/(lambda+mu) at the
// cells, 1/h per axis.
struct OpArgs {
    Dims dc;                     // cells
    Dims df[3];                  // face grids
    const double* w[3][3];       // w[a][axis]
    const c128* D[3];
    const double* C;
    double ih[3];
    int64_t off[4];              // field offsets in a vector
};

// y = H x (all fields) in one launch over the grid of (n1+1) x (n2+1) (x
// (n3+1)) points: the thread at (i, j, k) owns the a-face (i, j, k) of every
// face grid that has it and the cell (i, j, k) if it exists, keeps their
// coefficients in registers for the whole batch, and reads each right-hand
// side's u_a around its faces once: the same values give the stencil of A_a
// and the divergence of its cell.  Rows of u_a: A_a u_a + B_a^T p with
// B_a^T p = (p(c) - p(c - e_a)) / h_a (zero ghost p); rows of p:
// -sum_a (u_a(c + e_a) - u_a(c)) / h_a - p / (lambda + mu).
//
// Launch: blockDim 256 (OTX x OTY points), gridDim (x tiles, y tiles,
// planes x chunks of the batch); workgroup z takes plane z % planes and
// right-hand sides [c * rch, min(nrhs, c * rch + rch)) with c = z / planes.

// 2D, several right-hand sides per workgroup, each right-hand side's inputs
// staged in LDS.  A workgroup owns OTX x OTY points of the (n1+1) x (n2+1)
// grid; per right-hand side it
// loads the u_1 and u_2 faces of its box plus one point around it and the p
// cells of its box plus one below and to the left -- every value once,
// coalesced along x -- into one of two LDS buffers, and the next right-hand
// side's into registers while this one is computed from LDS: one barrier
// per right-hand side.  Values outside a field are zero (the zero ghosts of
// the operator).
//
// DOTS: the launch also does the first Gram-Schmidt pass of the Arnoldi
// step on the vector it writes, w = H z: for the stored basis columns
// t < J it forms, per right-hand side and workgroup, the partial sums
// conj(V_t) . w and conj(V_t) . V_{J-1} over the workgroup's degrees of
// freedom (each thread's faces and cell, then the wavefront butterfly, then
// the four wavefronts in a fixed order), so w need not be read back for
// them.  Partials [r][2J][workgroup]; k_reduce_partials adds them in a fixed
// order.
struct DotArgs {
    const c128* V;       // basis: column t of RHS r at V + t * vstep + r * (the output stride)
    int64_t vstep;
    int J;               // columns 0 .. J-1 (J <= KRY_MAXM)
    c128* partial;
};

constexpr int OTX = 64, OTY = 4;
constexpr int OP_MAXJ = 32;

// The DOTS epilogue for right-hand side r: the thread's NE degrees of
// freedom (has[e], at index at[e] within a vector) with w values yk[e];
// writes the workgroup's partials for columns t < J at workgroup index blk
// of nt.  Called by every thread of the workgroup (two barriers).
template <int NE>
__device__ __forceinline__ void gs_first_pass(const DotArgs& da, int r, int64_t vs, const bool* has,
                                              const int64_t* at, const c128* yk, int64_t blk, int64_t nt) {
    __shared__ double red[4][4 * OP_MAXJ];
    const int tid = threadIdx.x;
    const int J = da.J;
    const int lane = tid & 63, wave = tid >> 6;
    const c128* Vl = da.V + (int64_t)(J - 1) * da.vstep + r * vs;
    c128 vl[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) vl[e] = has[e] ? Vl[at[e]] : mk(0.0, 0.0);
    for (int t = 0; t < J; ++t) {
        const c128* Vt = da.V + (int64_t)t * da.vstep + r * vs;
        double ar = 0.0, ai = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const c128 v = t == J - 1 ? vl[e] : (has[e] ? Vt[at[e]] : mk(0.0, 0.0));
            ar += v.re * yk[e].re + v.im * yk[e].im;
            ai += v.re * yk[e].im - v.im * yk[e].re;
            gr += v.re * vl[e].re + v.im * vl[e].im;
            gi += v.re * vl[e].im - v.im * vl[e].re;
        }
        for (int off = 32; off > 0; off >>= 1) {
            ar += __shfl_xor(ar, off, 64);
            ai += __shfl_xor(ai, off, 64);
            gr += __shfl_xor(gr, off, 64);
            gi += __shfl_xor(gi, off, 64);
        }
        if (lane == 0) {
            red[wave][4 * t] = ar;
            red[wave][4 * t + 1] = ai;
            red[wave][4 * t + 2] = gr;
            red[wave][4 * t + 3] = gi;
        }
    }
    __syncthreads();
    if (tid < 2 * J) {
        const int t = tid % J, g = tid / J;   // g = 0: conj(V_t) w, 1: conj(V_t) V_{J-1}
        const int q = 4 * t + 2 * g;
        const double sr = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
        const double si = (red[0][q + 1] + red[1][q + 1]) + (red[2][q + 1] + red[3][q + 1]);
        da.partial[((int64_t)r * 2 * J + g * J + t) * nt + blk] = mk(sr, si);
    }
    __syncthreads();   // red is reused by the next right-hand side
}
template <class Tin, bool RES, bool DOTS = false>
__global__ void __launch_bounds__(256)
k_op2_lds(OpArgs o, const cplx<Tin>* __restrict__ x, c128* __restrict__ y, int nrhs, int64_t vs_in, int64_t vs_out,
          ResArgs ra, int rch, DotArgs da = DotArgs{}) {
    constexpr int UW = OTX + 2, UH = OTY + 2;        // u_a box: [x0-1, x0+OTX] x [y0-1, y0+OTY]
    constexpr int PW = OTX + 1, PH = OTY + 1;        // p box:   [x0-1, x0+OTX-1] x [y0-1, y0+OTY-1]
    constexpr int NU = UW * UH, NP = PW * PH, NS = 2 * NU + NP;
    constexpr int NR = (NS + 255) / 256;
    __shared__ cplx<Tin> lds[2][NS];
    const int tid = threadIdx.x;
    const int tx = tid % OTX, ty = tid / OTX;
    const int x0 = blockIdx.x * OTX, y0 = blockIdx.y * OTY;
    const int i = x0 + tx, j = y0 + ty;
    const int rlo = blockIdx.z * rch, rhi = min(nrhs, rlo + rch);
    const int n0 = o.dc.g[0], n1 = o.dc.g[1];
    const bool inx = i <= n0 && j <= n1;
    // staged entries of this thread: field offset + index, or -1 (zero)
    int64_t sidx[NR];
#pragma unroll
    for (int it = 0; it < NR; ++it) {
        const int q = tid + it * 256;
        int64_t v = -1;
        if (q < 2 * NU) {
            const int a = q / NU, e = q - a * NU;
            const int ey = e / UW, ex = e - ey * UW;
            const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            const Dims& d = o.df[a];
            if (gx >= 0 && gx < d.g[0] && gy >= 0 && gy < d.g[1]) v = o.off[a] + (int64_t)gy * d.g[0] + gx;
        } else if (q < NS) {
            const int e = q - 2 * NU;
            const int ey = e / PW, ex = e - ey * PW;
            const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            if (gx >= 0 && gx < n0 && gy >= 0 && gy < n1) v = o.off[2] + (int64_t)gy * n0 + gx;
        }
        sidx[it] = v;
    }
    // own faces and cell, coefficients for the whole batch
    bool face[2];
    int64_t fp[2];
    FineCoef<double, 0, 2> cf[2];
    c128 Dp[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const Dims& d = o.df[a];
        face[a] = inx && (a == 0 ? j < n1 : i < n0);
        fp[a] = (int64_t)j * d.g[0] + i;
        Dp[a] = mk(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < 3; ++b) { cf[a].cp[b] = 0.0; cf[a].cm[b] = 0.0; }
        if (face[a]) {
            cf[a].load(d, i, j, 0, fp[a], o.w[a][0], o.w[a][1], o.w[a][2], 0.0, 0.0, 0.0);
            Dp[a] = o.D[a][fp[a]];
        }
    }
    const bool cell = inx && i < n0 && j < n1;
    const int64_t pc = (int64_t)j * n0 + i;
    const double Cp = cell ? o.C[pc] : 0.0;
    // LDS positions of the own point in the u box (+1, +1) and the p box (+1, +1)
    const int lu = (ty + 1) * UW + (tx + 1);
    const int lp = 2 * NU + (ty + 1) * PW + (tx + 1);
    cplx<Tin> vin[NR];
    auto load_in = [&](int r) {
        const cplx<Tin>* xr = x + r * vs_in;
#pragma unroll
        for (int it = 0; it < NR; ++it) vin[it] = xr[sidx[it] >= 0 ? sidx[it] : 0];
    };
    load_in(rlo);
    for (int r = rlo; r < rhi; ++r) {
        cplx<Tin>* S = lds[(r - rlo) & 1];
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            const int q = tid + it * 256;
            if (q < NS) S[q] = sidx[it] >= 0 ? vin[it] : cplx<Tin>{Tin(0), Tin(0)};
        }
        if (r + 1 < rhi) load_in(r + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        double rr = 0.0;
        const c128 pcv = ccast<double>(S[lp]);
        c128 div = mk(0.0, 0.0);
        c128 yk[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};   // w at the faces and the cell
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (!face[a]) continue;
            const cplx<Tin>* U = S + a * NU;
            const c128 uc = ccast<double>(U[lu]);
            const c128 up[2] = {ccast<double>(U[lu + 1]), ccast<double>(U[lu + UW])};
            const c128 um[2] = {ccast<double>(U[lu - 1]), ccast<double>(U[lu - UW])};
            if (cell) div = div + o.ih[a] * (up[a] - uc);
            c128 sum = mk(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < 2; ++b) sum = sum + cf[a].cp[b] * up[b] + cf[a].cm[b] * um[b];
            // p at the cells on both sides of the face (zero ghost outside)
            const c128 g = pcv - ccast<double>(S[lp - (a == 0 ? 1 : PW)]);
            c128 yv = Dp[a] * uc - sum + o.ih[a] * g;
            if (RES) {
                yv = ra.b[r * vs_out + o.off[a] + fp[a]] - yv;
                rr += yv.re * yv.re + yv.im * yv.im;
            }
            y[r * vs_out + o.off[a] + fp[a]] = yv;
            yk[a] = yv;
        }
        if (cell) {
            c128 yv = mk(-div.re - Cp * pcv.re, -div.im - Cp * pcv.im);
            if (RES) {
                yv = ra.b[r * vs_out + o.off[2] + pc] - yv;
                rr += yv.re * yv.re + yv.im * yv.im;
            }
            y[r * vs_out + o.off[2] + pc] = yv;
            yk[2] = yv;
        }
        if (RES) res_partial(ra, r, 0, rr);
        if (DOTS) {
            const bool has[3] = {face[0], face[1], cell};
            const int64_t at[3] = {o.off[0] + fp[0], o.off[1] + fp[1], o.off[2] + pc};
            const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
            gs_first_pass<3>(da, r, vs_out, has, at, yk, blk, (int64_t)gridDim.x * gridDim.y);
        }
    }
}

// 3D, several right-hand sides per workgroup, each right-hand side's plane
// staged in LDS.  A workgroup owns OTX x OTY points of plane k of the
// (n1+1) x (n2+1) x (n3+1) grid; per right-hand side it stages u_1, u_2, u_3 at plane k over its
// box plus one point around it and p at plane k over its box plus one
// below and to the left -- every value once, coalesced along x -- into one
// of two LDS buffers, and loads the values one plane below and above that
// the z-stencils, the z-face pressure difference and the divergence need
// (u_a at k-1 and k+1 of the own faces, p at k-1 of the own cell) straight
// from memory; the next right-hand side's loads are in flight while this
// one is computed.  One barrier per right-hand side.
template <class Tin, bool RES>
__global__ void __launch_bounds__(256)
k_op3_lds(OpArgs o, const cplx<Tin>* __restrict__ x, c128* __restrict__ y, int nrhs, int64_t vs_in, int64_t vs_out,
          ResArgs ra, int rch) {
    constexpr int UW = OTX + 2, UH = OTY + 2;
    constexpr int PW = OTX + 1, PH = OTY + 1;
    constexpr int NU = UW * UH, NP = PW * PH, NS = 3 * NU + NP;
    constexpr int NR = (NS + 255) / 256;
    __shared__ cplx<Tin> lds[2][NS];
    const int tid = threadIdx.x;
    const int tx = tid % OTX, ty = tid / OTX;
    const int x0 = blockIdx.x * OTX, y0 = blockIdx.y * OTY;
    const int i = x0 + tx, j = y0 + ty;
    const int n0 = o.dc.g[0], n1 = o.dc.g[1], n2 = o.dc.g[2];
    const int planes = n2 + 1;
    const int k = blockIdx.z % planes;
    const int rlo = (blockIdx.z / planes) * rch, rhi = min(nrhs, rlo + rch);
    const bool inx = i <= n0 && j <= n1;
    int64_t sidx[NR];
#pragma unroll
    for (int it = 0; it < NR; ++it) {
        const int q = tid + it * 256;
        int64_t v = -1;
        if (q < 3 * NU) {
            const int a = q / NU, e = q - a * NU;
            const int ey = e / UW, ex = e - ey * UW;
            const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            const Dims& d = o.df[a];
            if (gx >= 0 && gx < d.g[0] && gy >= 0 && gy < d.g[1] && k < d.g[2])
                v = o.off[a] + ((int64_t)k * d.g[1] + gy) * d.g[0] + gx;
        } else if (q < NS) {
            const int e = q - 3 * NU;
            const int ey = e / PW, ex = e - ey * PW;
            const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            if (gx >= 0 && gx < n0 && gy >= 0 && gy < n1 && k < n2)
                v = o.off[3] + ((int64_t)k * n1 + gy) * n0 + gx;
        }
        sidx[it] = v;
    }
    const int ci[3] = {i, j, k};
    const int nn[3] = {n0, n1, n2};
    bool face[3];
    int64_t fp[3], fsz[3];
    FineCoef<double, 0, 3> cf[3];
    c128 Dp[3];
    bool zm[3], zp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const Dims& d = o.df[a];
        bool ok = inx;
#pragma unroll
        for (int b = 0; b < 3; ++b) if (b != a && ci[b] >= nn[b]) ok = false;
        face[a] = ok;
        fsz[a] = (int64_t)d.g[0] * d.g[1];
        fp[a] = k * fsz[a] + (int64_t)j * d.g[0] + i;
        zm[a] = ok && k > 0;
        zp[a] = ok && k + 1 < d.g[2];
        Dp[a] = mk(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < 3; ++b) { cf[a].cp[b] = 0.0; cf[a].cm[b] = 0.0; }
        if (ok) {
            cf[a].load(d, i, j, k, fp[a], o.w[a][0], o.w[a][1], o.w[a][2], 0.0, 0.0, 0.0);
            Dp[a] = o.D[a][fp[a]];
        }
    }
    const bool cell = inx && i < n0 && j < n1 && k < n2;
    const int64_t csz = (int64_t)n0 * n1;
    const int64_t pc = k * csz + (int64_t)j * n0 + i;
    const bool pzm = face[2] && k > 0;     // p in the cell below the own z-face
    const double Cp = cell ? o.C[pc] : 0.0;
    const int lu = (ty + 1) * UW + (tx + 1);
    const int lp = 3 * NU + (ty + 1) * PW + (tx + 1);
    cplx<Tin> vin[NR];
    cplx<Tin> vzm[3], vzp[3], vpm;
    auto load_in = [&](int r) {
        const cplx<Tin>* xr = x + r * vs_in;
#pragma unroll
        for (int it = 0; it < NR; ++it) vin[it] = xr[sidx[it] >= 0 ? sidx[it] : 0];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cplx<Tin>* ur = xr + o.off[a];
            vzm[a] = ur[zm[a] ? fp[a] - fsz[a] : 0];
            vzp[a] = ur[zp[a] ? fp[a] + fsz[a] : 0];
        }
        vpm = xr[o.off[3] + (pzm ? pc - csz : 0)];
    };
    load_in(rlo);
    for (int r = rlo; r < rhi; ++r) {
        cplx<Tin>* S = lds[(r - rlo) & 1];
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            const int q = tid + it * 256;
            if (q < NS) S[q] = sidx[it] >= 0 ? vin[it] : cplx<Tin>{Tin(0), Tin(0)};
        }
        c128 um2[3], up2[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            um2[a] = zm[a] ? ccast<double>(vzm[a]) : mk(0.0, 0.0);
            up2[a] = zp[a] ? ccast<double>(vzp[a]) : mk(0.0, 0.0);
        }
        const c128 pm2 = pzm ? ccast<double>(vpm) : mk(0.0, 0.0);
        if (r + 1 < rhi) load_in(r + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        double rr = 0.0;
        const c128 pcv = ccast<double>(S[lp]);
        c128 div = mk(0.0, 0.0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (!face[a]) continue;
            const cplx<Tin>* U = S + a * NU;
            const c128 uc = ccast<double>(U[lu]);
            const c128 up[3] = {ccast<double>(U[lu + 1]), ccast<double>(U[lu + UW]), up2[a]};
            const c128 um[3] = {ccast<double>(U[lu - 1]), ccast<double>(U[lu - UW]), um2[a]};
            if (cell) div = div + o.ih[a] * (up[a] - uc);
            c128 s = mk(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < 3; ++b) s = s + cf[a].cp[b] * up[b] + cf[a].cm[b] * um[b];
            // p at the cells on both sides of the face (zero ghost outside)
            const c128 pnb = a == 2 ? pm2 : ccast<double>(S[lp - (a == 0 ? 1 : PW)]);
            const c128 g = pcv - pnb;
            c128 yv = Dp[a] * uc - s + o.ih[a] * g;
            if (RES) {
                yv = ra.b[r * vs_out + o.off[a] + fp[a]] - yv;
                rr += yv.re * yv.re + yv.im * yv.im;
            }
            y[r * vs_out + o.off[a] + fp[a]] = yv;
        }
        if (cell) {
            c128 yv = mk(-div.re - Cp * pcv.re, -div.im - Cp * pcv.im);
            if (RES) {
                yv = ra.b[r * vs_out + o.off[3] + pc] - yv;
                rr += yv.re * yv.re + yv.im * yv.im;
            }
            y[r * vs_out + o.off[3] + pc] = yv;
        }
        if (RES) res_partial(ra, r, k, rr);
    }
}

// TILDE: the Remark's A~_p r = B A_f(mu) B^T r - w^2 rho (1 - i gamma/w) r,
// sum over faces of mu_f (r_c - r_nb) / h_a^2 with mu_f the mean over the
// face's existing cells and r = 0 beyond the boundary.
template <class T, int DIM, bool TILDE>
__global__ void __launch_bounds__(256)
k_distribute(Dims dc, const c128* __restrict__ r0, const c128* __restrict__ r1,
             const c128* __restrict__ r2, const c128* __restrict__ rp,
             const double* __restrict__ mu, const c128* __restrict__ mcell, double om2,
             double ih0, double ih1, double ih2, cplx<T>* __restrict__ t, int nrhs,
             int64_t vs_in, int64_t vs_out, const double* __restrict__ rs, int64_t rss, int rch) {
    // grid z: planes x chunks of the batch, as for the operator kernels
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z % dc.g[2];
    const int rlo = (blockIdx.z / dc.g[2]) * rch, rhi = min(nrhs, rlo + rch);
    if (i >= dc.g[0] || j >= dc.g[1]) return;
    const int64_t sy = dc.g[0], sz = (int64_t)dc.g[0] * dc.g[1];
    const int64_t p = k * sz + j * sy + i;
    const int64_t f0 = ((int64_t)k * dc.g[1] + j) * (dc.g[0] + 1) + i;
    const int64_t f1 = ((int64_t)k * (dc.g[1] + 1) + j) * dc.g[0] + i;
    const int64_t f2 = ((int64_t)k * dc.g[1] + j) * dc.g[0] + i;
    const int64_t s2 = (int64_t)dc.g[0] * dc.g[1];
    const double ihs[3] = {ih0 * ih0, ih1 * ih1, ih2 * ih2};
    const int64_t st[3] = {1, sy, sz};
    const int ci[3] = {i, j, k};
    const double mup = mu[p];
    double mnb[3][2];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        mnb[a][0] = (ci[a] > 0) ? mu[p - st[a]] : 0.0;
        mnb[a][1] = (ci[a] + 1 < dc.g[a]) ? mu[p + st[a]] : 0.0;
    }
    const c128 mc = mcell[p];
    for (int r = rlo; r < rhi; ++r) {
        const int64_t o = r * vs_in;
        c128 div = ih0 * (r0[o + f0 + 1] - r0[o + f0]);
        div = div + ih1 * (r1[o + f1 + dc.g[0]] - r1[o + f1]);
        if (DIM == 3) div = div + ih2 * (r2[o + f2 + s2] - r2[o + f2]);
        const c128* pr = rp + o;
        const c128 pc = pr[p];
        c128 lap = mk(0.0, 0.0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            c128 s;
            if (TILDE) {
                // B A_f(mu) B^T r: sum over the two faces along a
                const bool lo = ci[a] > 0, hi = ci[a] + 1 < dc.g[a];
                const double mlo = lo ? 0.5 * (mup + mnb[a][0]) : mup;
                const double mhi = hi ? 0.5 * (mup + mnb[a][1]) : mup;
                s = (mlo + mhi) * pc;
                if (lo) s = s - mlo * pr[p - st[a]];
                if (hi) s = s - mhi * pr[p + st[a]];
            } else {
                // B B^T (mu r): sum_a (2 mu_c r_c - mu_c+ r_c+ - mu_c- r_c-) / h_a^2
                s = (2.0 * mup) * pc;
                if (ci[a] > 0) s = s - mnb[a][0] * pr[p - st[a]];
                if (ci[a] + 1 < dc.g[a]) s = s - mnb[a][1] * pr[p + st[a]];
            }
            lap = lap + ihs[a] * s;
        }
        const c128 Apr = lap - om2 * (mc * pc);
        const double sr = rs ? rs[r * rss] : 1.0;
        const c128 tv = mk(sr * (-div.re - Apr.re), sr * (-div.im - Apr.im));
        t[r * vs_out + p] = ccast<T>(tv);
    }
}

// out[q * vo + i] = s_q in[q * vi + i] in the output precision, s_q =
// rs[q * rss] (1 without rs); one grid row per right-hand side
template <class To>
__global__ void __launch_bounds__(256)
k_cast_scaled(int64_t n, const c128* __restrict__ in, int64_t vi, const double* __restrict__ rs, int64_t rss,
              cplx<To>* __restrict__ out, int64_t vo) {
    const int q = blockIdx.y;
    const double sq = rs ? rs[q * rss] : 1.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[q * vo + i] = ccast<To>(sq * in[q * vi + i]);
}

// out = s * in (the power method's normalisation)
__global__ void __launch_bounds__(256)
k_scal(int64_t n, double s, const c128* __restrict__ in, c128* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) out[p] = s * in[p];
}

template <class To, class Ti>
__global__ void __launch_bounds__(256)
k_cast(int64_t n, const cplx<Ti>* __restrict__ in, cplx<To>* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = t; q < n; q += stride) out[q] = ccast<To>(in[q]);
}

}  // namespace eh
