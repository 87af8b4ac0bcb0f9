// 3D intergrid transfers (Section 4.5) with the values a tile needs staged
// in LDS: prolongation with correction u += P e (trilinear interpolation)
// and restriction f_c = R r (full weighting, or the mixed restriction of
// eq. tildeRu1).
//
// Prolongation.  A workgroup owns PTX x PTY points of fine plane k of one
// block.  Along z the plane takes the same two coarse planes and weights for
// all its points, so per right-hand side the workgroup loads the coarse entries
// its tile interpolates from (PTX / 2 + 2 by PTY / 2 + 2 per coarse plane,
// coalesced along x), interpolates them in z once into one of two LDS
// buffers and loads the next right-hand side's coarse entries and u while
// this one is computed: one barrier per right-hand side.  Each point then
// interpolates in y of x from LDS and updates its u in place.
//
// Per axis a fine index l takes coarse indices and weights as p1 gives
// them: nodal axes l / 2 (weight 1) or (l - 1) / 2 and (l + 1) / 2 (1/2
// each); cell-centred axes l / 2 (3/4) and its neighbour towards l (1/4,
// none at the boundary).
//
// Grid: (x tiles, y tiles, maxg2 * ns * chunks) over the fine grids (d[]),
// coarse grids in dc[]; workgroup z takes plane z % maxg2 of slot
// (z / maxg2) % ns and the chunk z / (maxg2 * ns) of rch right-hand sides.
//
// Restriction.  A workgroup owns RTX x RTY points of coarse plane K.  Along
// an axis coarse index I takes the fine indices 2I + FIRST .. 2I + FIRST +
// S - 1 with the weights of R1 (nodal: 1/4, 1/2, 1/4 around 2I; cell-
// centred full weighting 1/8, 3/8, 3/8, 1/8 from 2I - 1; mixed cell-centred
// 1/2, 1/2 from 2I), so a tile's fine box is 2 RTX + 2 by 2 RTY + 2 columns
// from (2 x0 - 1, 2 y0 - 1) on the S_z planes of K.  Per right-hand side
// the workgroup loads every column of the box on those planes (coalesced
// along x), sums each column in z with the z weights into one of two LDS
// buffers and loads the next right-hand side's columns while this one is
// computed; each coarse point then sums its S_x x S_y columns from LDS.
// Fine values outside the grid are zero.  Grid: (x tiles, y tiles, maxg2 *
// ns * chunks) over the coarse grids (d[]), fine grids in dc[].
#pragma once

#include "eh_common.h"
#include "eh_group_kernels.h"
#include "eh_mg_kernels.h"

namespace eh {

constexpr int PTX = 32, PTY = 8;
constexpr int PCW = PTX / 2 + 2, PCH = PTY / 2 + 2, PNC = PCW * PCH;

template <class T, int NM>
__device__ __forceinline__ void prolong3_body(const GArgs<T>& a, int slot, int k, int rlo, int rhi,
                                              cplx<T> (&lds)[2][PNC]) {
    const Dims df = a.d[slot], dc = a.dc[slot];
    const int x0 = blockIdx.x * PTX, y0 = blockIdx.y * PTY;
    const int tid = threadIdx.x;
    const int i = x0 + tid % PTX, j = y0 + tid / PTX;
    const bool mine = i < df.g[0] && j < df.g[1];
    int zi0, zi1;
    float zw0, zw1;
    p1<(NM & 4) != 0>(k, dc.g[2], zi0, zi1, zw0, zw1);
    // the coarse box of the tile starts one entry before the coarse index
    // of its first fine point
    const int cx0 = (x0 >> 1) - 1, cy0 = (y0 >> 1) - 1;
    const int gx = cx0 + tid % PCW, gy = cy0 + tid / PCW;
    const bool stg = tid < PNC && gx >= 0 && gx < dc.g[0] && gy >= 0 && gy < dc.g[1];
    const int64_t csz = (int64_t)dc.g[0] * dc.g[1];
    const int64_t q0 = stg ? (int64_t)zi0 * csz + (int64_t)gy * dc.g[0] + gx : 0;
    const int64_t q1 = stg ? (int64_t)zi1 * csz + (int64_t)gy * dc.g[0] + gx : 0;
    int xi[2], yi[2];
    float xw[2], yw[2];
    p1<(NM & 1) != 0>(mine ? i : 0, dc.g[0], xi[0], xi[1], xw[0], xw[1]);
    p1<(NM & 2) != 0>(mine ? j : 0, dc.g[1], yi[0], yi[1], yw[0], yw[1]);
    // local offsets in the staged box (in [0, PCW) x [0, PCH) for own points)
    const int l00 = (yi[0] - cy0) * PCW + (xi[0] - cx0), l01 = (yi[0] - cy0) * PCW + (xi[1] - cx0);
    const int l10 = (yi[1] - cy0) * PCW + (xi[0] - cx0), l11 = (yi[1] - cy0) * PCW + (xi[1] - cx0);
    const T tz0 = T(zw0), tz1 = T(zw1), tx0 = T(xw[0]), tx1 = T(xw[1]), ty0 = T(yw[0]), ty1 = T(yw[1]);
    const int64_t p = mine ? (int64_t)k * df.g[0] * df.g[1] + (int64_t)j * df.g[0] + i : 0;
    const cplx<T>* __restrict__ ec = a.f[slot];
    const int64_t vc = a.vf[slot];
    cplx<T>* __restrict__ u = a.out[slot];
    const int64_t vu = a.vo[slot];
    cplx<T> e0, e1, uv;
    auto load_in = [&](int r) {
        e0 = ec[(int64_t)r * vc + q0];
        e1 = ec[(int64_t)r * vc + q1];
        uv = u[(int64_t)r * vu + p];
    };
    if (rlo < rhi) load_in(rlo);
    for (int r = rlo; r < rhi; ++r) {
        cplx<T>* S = lds[(r - rlo) & 1];
        if (tid < PNC)
            S[tid] = stg ? mk<T>(fmat(tz1, e1.re, tz0 * e0.re), fmat(tz1, e1.im, tz0 * e0.im)) : czero<T>();
        const cplx<T> ur = uv;
        if (r + 1 < rhi) load_in(r + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (!mine) continue;
        const cplx<T> c00 = S[l00], c01 = S[l01], c10 = S[l10], c11 = S[l11];
        const cplx<T> r0 = mk<T>(fmat(tx1, c01.re, tx0 * c00.re), fmat(tx1, c01.im, tx0 * c00.im));
        const cplx<T> r1 = mk<T>(fmat(tx1, c11.re, tx0 * c10.re), fmat(tx1, c11.im, tx0 * c10.im));
        const cplx<T> s = mk<T>(fmat(ty1, r1.re, ty0 * r0.re), fmat(ty1, r1.im, ty0 * r0.im));
        u[(int64_t)r * vu + p] = ur + s;
    }
}

template <class T>
__global__ void __launch_bounds__(256)
k_gprolong3_lds(GArgs<T> a, int nrhs, int rch) {
    __shared__ cplx<T> lds[2][PNC];
    const int zq = blockIdx.z / a.maxg2;
    const int k = blockIdx.z - zq * a.maxg2;
    const int slot = zq % a.ns;
    const int rlo = (zq / a.ns) * rch, rhi = min(nrhs, rlo + rch);
    const Dims d = a.d[slot];
    if (k >= d.g[2] || (int)blockIdx.x * PTX >= d.g[0] || (int)blockIdx.y * PTY >= d.g[1]) return;   // uniform
    const int kind = a.kind[slot];
    if (kind == 3) prolong3_body<T, 0>(a, slot, k, rlo, rhi, lds);
    else if (kind == 0) prolong3_body<T, 1>(a, slot, k, rlo, rhi, lds);
    else if (kind == 1) prolong3_body<T, 2>(a, slot, k, rlo, rhi, lds);
    else prolong3_body<T, 4>(a, slot, k, rlo, rhi, lds);
}

constexpr int RTX = 32, RTY = 8;
constexpr int RBW = 2 * RTX + 2, RBH = 2 * RTY + 2, RNB = RBW * RBH;
constexpr int RNR = (RNB + 255) / 256;

template <class T, int NM, bool MIXED>
__device__ __forceinline__ void restrict3_body(const GArgs<T>& a, int slot, int K, int rlo, int rhi,
                                               cplx<T> (&lds)[2][RNB]) {
    using RX = R1<(NM & 1) != 0, MIXED>;
    using RY = R1<(NM & 2) != 0, MIXED>;
    using RZ = R1<(NM & 4) != 0, MIXED>;
    const Dims dcs = a.d[slot], df = a.dc[slot];
    const int x0 = blockIdx.x * RTX, y0 = blockIdx.y * RTY;
    const int tid = threadIdx.x;
    const int I = x0 + tid % RTX, J = y0 + tid / RTX;
    const bool mine = I < dcs.g[0] && J < dcs.g[1];
    const int fx0 = 2 * x0 - 1, fy0 = 2 * y0 - 1;
    const int64_t fsy = df.g[0], fsz = (int64_t)df.g[0] * df.g[1];
    int64_t col[RNR];
#pragma unroll
    for (int it = 0; it < RNR; ++it) {
        const int q = tid + it * 256;
        const int ey = q / RBW, ex = q - ey * RBW;
        const int gx = fx0 + ex, gy = fy0 + ey;
        col[it] = (q < RNB && gx >= 0 && gx < df.g[0] && gy >= 0 && gy < df.g[1]) ? (int64_t)gy * fsy + gx : -1;
    }
    const int z0 = 2 * K + RZ::FIRST;
    int64_t zoff[RZ::S];
    bool zok[RZ::S];
#pragma unroll
    for (int aa = 0; aa < RZ::S; ++aa) {
        zok[aa] = z0 + aa >= 0 && z0 + aa < df.g[2];
        zoff[aa] = zok[aa] ? (int64_t)(z0 + aa) * fsz : 0;
    }
    // this point's first column in the box
    const int lb = (2 * (J - y0) + RY::FIRST + 1) * RBW + 2 * (I - x0) + RX::FIRST + 1;
    const int64_t P = mine ? (int64_t)K * dcs.g[0] * dcs.g[1] + (int64_t)J * dcs.g[0] + I : 0;
    const cplx<T>* __restrict__ rf = a.f[slot];
    const int64_t vf = a.vf[slot];
    cplx<T>* __restrict__ fc = a.out[slot];
    const int64_t vo = a.vo[slot];
    cplx<T> v[RNR][RZ::S];
    auto load_in = [&](int r) {
        const cplx<T>* src = rf + (int64_t)r * vf;
#pragma unroll
        for (int it = 0; it < RNR; ++it)
#pragma unroll
            for (int aa = 0; aa < RZ::S; ++aa) v[it][aa] = src[zoff[aa] + (col[it] >= 0 ? col[it] : 0)];
    };
    if (rlo < rhi) load_in(rlo);
    for (int r = rlo; r < rhi; ++r) {
        cplx<T>* S = lds[(r - rlo) & 1];
#pragma unroll
        for (int it = 0; it < RNR; ++it) {
            const int q = tid + it * 256;
            if (q < RNB) {
                cplx<T> c = czero<T>();
#pragma unroll
                for (int aa = 0; aa < RZ::S; ++aa) {
                    const T wz = (zok[aa] && col[it] >= 0) ? T(RZ::w(aa)) : T(0);
                    c = mk<T>(fmat(wz, v[it][aa].re, c.re), fmat(wz, v[it][aa].im, c.im));
                }
                S[q] = c;
            }
        }
        if (r + 1 < rhi) load_in(r + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (!mine) continue;
        cplx<T> s = czero<T>();
#pragma unroll
        for (int b = 0; b < RY::S; ++b) {
            cplx<T> t = czero<T>();
#pragma unroll
            for (int cc = 0; cc < RX::S; ++cc) {
                const cplx<T> c = S[lb + b * RBW + cc];
                t = mk<T>(fmat(T(RX::w(cc)), c.re, t.re), fmat(T(RX::w(cc)), c.im, t.im));
            }
            s = mk<T>(fmat(T(RY::w(b)), t.re, s.re), fmat(T(RY::w(b)), t.im, s.im));
        }
        fc[(int64_t)r * vo + P] = s;
    }
}

template <class T, bool MIXED>
__global__ void __launch_bounds__(256)
k_grestrict3_lds(GArgs<T> a, int nrhs, int rch) {
    __shared__ cplx<T> lds[2][RNB];
    const int zq = blockIdx.z / a.maxg2;
    const int K = blockIdx.z - zq * a.maxg2;
    const int slot = zq % a.ns;
    const int rlo = (zq / a.ns) * rch, rhi = min(nrhs, rlo + rch);
    const Dims d = a.d[slot];
    if (K >= d.g[2] || (int)blockIdx.x * RTX >= d.g[0] || (int)blockIdx.y * RTY >= d.g[1]) return;   // uniform
    const int kind = a.kind[slot];
    if (kind == 3) restrict3_body<T, 0, MIXED>(a, slot, K, rlo, rhi, lds);
    else if (kind == 0) restrict3_body<T, 1, MIXED>(a, slot, K, rlo, rhi, lds);
    else if (kind == 1) restrict3_body<T, 2, MIXED>(a, slot, K, rlo, rhi, lds);
    else restrict3_body<T, 4, MIXED>(a, slot, K, rlo, rhi, lds);
}

}  // namespace eh
