// Multigrid kernels over a group of acoustic blocks in one launch.
//
// The shear blocks A_1..A_d of the preconditioner are independent (the
// block-diagonal A of eq. prec), so each stage of their cycles -- a Jacobi
// sweep, a residual, a restriction, a prolongation, the coarsest solve --
// runs for all of them in a single launch: blockIdx.z enumerates
// (slot, z-plane) pairs and every workgroup serves one block.  The pressure
// block H_p runs as a group of one.  The per-block stencil shape is chosen
// at compile time by a switch that is uniform across a workgroup.
//
// Modes of the sweep kernels:
//   0  out = w D^-1 f                          (first sweep, zero guess)
//   1  out = u + w D^-1 (f - X u)              (damped Jacobi)
//   2  out = f - X u                           (residual)
//   3  out = X u                               (operator)
//   4  out = w D^-1 f and out2 = f - X out     (first sweep fused with the
//      residual: the neighbours' w D^-1 f is recomputed from f and D)
//   5  out = u1 + w D^-1 (f - X u1), u1 = w D^-1 f (the first two sweeps
//      from a zero guess in one pass, u1 of the neighbours recomputed)
#pragma once

#include "eh_common.h"
#include "eh_mg_kernels.h"

namespace eh {

constexpr int GMAX = 3;

template <class T>
struct GArgs {
    int ns;                  // slots in use
    int kind[GMAX];          // block per slot: 0..dim-1 = A_{k+1}, dim = H_p
    int maxg2;               // largest z extent among the slots
    Dims d[GMAX];            // grid of the level the kernel runs on
    Dims dc[GMAX];           // coarse grid (transfers)
    const cplx<T>* f[GMAX];
    const cplx<T>* u[GMAX];
    cplx<T>* out[GMAX];
    cplx<T>* out2[GMAX];
    int64_t vf[GMAX], vu[GMAX], vo[GMAX], vo2[GMAX];
    const T* w[GMAX][3];     // fine-level couplings
    const cplx<T>* D[GMAX];  // fine-level diagonal
    const cplx<T>* coef[GMAX];   // coarse-level stencil
    const cplx<T>* dinv[GMAX];   // coarse level: damping / diagonal per point
    T damp;
    T ih[3];                 // 1 / h_a^2
    int mixed;               // mixed intergrid (27-point coarse stencils)
    int tilde;               // H_p built from A~_p (fine couplings of KIND 2)
};

// Grid: (x, y, maxg2 * ns * chunks).  Workgroup z covers plane k = z %
// maxg2 of slot (z / maxg2) % ns and right-hand sides [rlo, rhi), chunk
// z / (maxg2 * ns) of RCH each (RCH = nrhs: the whole batch).  Splitting a
// batch over workgroups changes only which workgroup computes a right-hand
// side, not its arithmetic.
#define EH_GROUP_POINT(a, DD, RCH)                                              \
    const int zq = blockIdx.z / (a).maxg2;                                      \
    const int k = blockIdx.z - zq * (a).maxg2;                                  \
    const int slot = zq % (a).ns;                                               \
    const int rlo = (zq / (a).ns) * (RCH), rhi = min(nrhs, rlo + (RCH));        \
    const Dims d = (a).DD[slot];                                                \
    if (k >= d.g[2]) return;                                                    \
    const int i = blockIdx.x * blockDim.x + threadIdx.x;                        \
    const int j = blockIdx.y * blockDim.y + threadIdx.y;                        \
    if (i >= d.g[0] || j >= d.g[1]) return;                                     \
    const int64_t sy = d.g[0], sz = (int64_t)d.g[0] * d.g[1];                   \
    const int64_t p = k * sz + j * sy + i;

// ---------------------------------------------------------------------------
// fine level (matrix-free)

template <class T, int KIND, int DIM, int MODE>
__global__ void __launch_bounds__(256)
k_gfine(GArgs<T> a, int nrhs, int rch) {
    EH_GROUP_POINT(a, d, rch)
    const T* __restrict__ w0 = a.w[slot][0];
    const T* __restrict__ w1 = a.w[slot][1];
    const T* __restrict__ w2 = a.w[slot][2];
    const cplx<T>* __restrict__ D = a.D[slot];
    const cplx<T>* __restrict__ f = a.f[slot];
    cplx<T>* __restrict__ out = a.out[slot];
    const int64_t vf = a.vf[slot], vo = a.vo[slot];
    const cplx<T> Dp = D[p];
    const T damp = a.damp;
    const cplx<T> sc = cdiv(mk<T>(damp, T(0)), Dp);
    if (MODE == 0) {
        for (int r = rlo; r < rhi; ++r) out[r * vo + p] = sc * f[r * vf + p];
        return;
    }
    FineCoef<T, KIND, DIM> c;
    c.load(d, i, j, k, p, w0, w1, w2, a.ih[0], a.ih[1], a.ih[2]);
    // neighbour offsets and couplings; a missing neighbour gets coupling 0
    // and the point's own offset
    constexpr int NN = 2 * DIM;
    int off[NN];
    cplx<T> cw[NN];
    {
        const int64_t st[3] = {1, sy, sz};
        const int ci[3] = {i, j, k};
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            const bool hm = ci[ax] > 0, hp = ci[ax] + 1 < d.g[ax];
            off[2 * ax] = hm ? -(int)st[ax] : 0;
            off[2 * ax + 1] = hp ? (int)st[ax] : 0;
            cw[2 * ax] = mk<T>(hm ? c.cm[ax] : T(0), T(0));
            cw[2 * ax + 1] = mk<T>(hp ? c.cp[ax] : T(0), T(0));
            if (MODE == 4 || MODE == 5) {
                // fold the neighbour's first-sweep factor damp / D_nb in
                cw[2 * ax] = cw[2 * ax] * (hm ? cdiv(mk<T>(damp, T(0)), D[p + off[2 * ax]]) : czero<T>());
                cw[2 * ax + 1] = cw[2 * ax + 1] * (hp ? cdiv(mk<T>(damp, T(0)), D[p + off[2 * ax + 1]]) : czero<T>());
            }
        }
    }
    if (MODE == 4 || MODE == 5) {
#pragma unroll 2
        for (int r = rlo; r < rhi; ++r) {
            const cplx<T>* __restrict__ fr = f + r * vf;
            const cplx<T> fp = fr[p];
            const cplx<T> u0 = sc * fp;
            cplx<T> s = czero<T>();
#pragma unroll
            for (int t = 0; t < NN; ++t) s = s + cw[t] * fr[p + off[t]];
            const cplx<T> r0 = fp - Dp * u0 + s;
            if (MODE == 4) {
                out[r * vo + p] = u0;
                a.out2[slot][r * a.vo2[slot] + p] = r0;
            } else {
                out[r * vo + p] = u0 + sc * r0;
            }
        }
        return;
    }
    const cplx<T>* __restrict__ u = a.u[slot];
    const int64_t vu = a.vu[slot];
#pragma unroll 2
    for (int r = rlo; r < rhi; ++r) {
        const cplx<T>* __restrict__ ur = u + r * vu;
        const cplx<T> up = ur[p];
        cplx<T> offs = czero<T>();
#pragma unroll
        for (int t = 0; t < NN; ++t) offs = offs + cw[t] * ur[p + off[t]];
        if (MODE == 1) {
            out[r * vo + p] = up + sc * (f[r * vf + p] - Dp * up + offs);
        } else if (MODE == 2) {
            out[r * vo + p] = f[r * vf + p] - Dp * up + offs;
        } else {
            out[r * vo + p] = Dp * up - offs;
        }
    }
}

// ---------------------------------------------------------------------------
// coarse levels (stored Galerkin stencils)

// Coefficient of stencil offset o at point p of a stored Galerkin stencil
// (offsets enumerated x fastest over a centrally symmetric box, so offset
// NST-1-o is the mirror of o).  The shear blocks A_k are complex symmetric
// and full weighting R = P^T / 2^d keeps that on every level, so for them
// (HALF) only the offsets o >= CENTRE are stored: offset o < CENTRE at p equals the
// mirrored offset stored at the neighbour q = p + offset(o), which the
// caller guarantees to lie in the grid.
template <class T, int NST, bool HALF>
__device__ __forceinline__ cplx<T> stencil_coef(const cplx<T>* __restrict__ coef, int64_t np, int o, int64_t p,
                                                int64_t q) {
    constexpr int C = NST / 2;
    if (!HALF) return coef[o * np + p];
    if (o >= C) return coef[(o - C) * np + p];
    return coef[(NST - 1 - o - C) * np + q];
}

// dinv = damping / centre coefficient, once per level at setup
template <class T, int CENTRE>
__global__ void k_dinv(int64_t np, const cplx<T>* __restrict__ coef, T damp, cplx<T>* __restrict__ dinv) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < np) dinv[p] = cdiv(mk<T>(damp, T(0)), coef[CENTRE * np + p]);
}

template <class T, int WX, int WY, int WZ, int MODE, bool HALF>
__device__ __forceinline__ void stencil_body(const GArgs<T>& a, int slot, const Dims& d, int i, int j, int k,
                                             int64_t p, int64_t sy, int64_t sz, int rlo, int rhi) {
    const int64_t np = d.np();
    constexpr int NX = 2 * WX + 1, NY = 2 * WY + 1, NZ = 2 * WZ + 1;
    constexpr int NST = NX * NY * NZ;
    const cplx<T>* __restrict__ coef = a.coef[slot];
    const cplx<T>* __restrict__ dinv = a.dinv[slot];
    const cplx<T>* __restrict__ f = a.f[slot];
    cplx<T>* __restrict__ out = a.out[slot];
    const int64_t vf = a.vf[slot], vo = a.vo[slot];
    const cplx<T> sc = dinv[p];
    if (MODE == 0) {
        for (int r = rlo; r < rhi; ++r) out[r * vo + p] = sc * f[r * vf + p];
        return;
    }
    const cplx<T>* __restrict__ u = a.u[slot];
    const int64_t vu = a.vu[slot];
    if (NST <= 27) {
        // stencil in registers; a missing neighbour gets a zero coefficient
        // and reads the point itself, so the batch loop has no branches and
        // every coefficient is read once per launch.  Neighbour offsets are
        // recomputed from the (uniform) strides rather than held per lane.
        cplx<T> cf[NST];
        unsigned okmask = 0;
#pragma unroll
        for (int oz = -WZ; oz <= WZ; ++oz)
#pragma unroll
            for (int oy = -WY; oy <= WY; ++oy)
#pragma unroll
                for (int ox = -WX; ox <= WX; ++ox) {
                    const int o = ((oz + WZ) * NY + (oy + WY)) * NX + (ox + WX);
                    const bool ok = (k + oz >= 0) && (k + oz < d.g[2]) && (j + oy >= 0) && (j + oy < d.g[1]) &&
                                    (i + ox >= 0) && (i + ox < d.g[0]);
                    okmask |= ok ? (1u << o) : 0u;
                    cf[o] = ok ? stencil_coef<T, NST, HALF>(coef, np, o, p, p + oz * sz + oy * sy + ox) : czero<T>();
                    if (MODE == 4 || MODE == 5) {
                        // neighbour's first-sweep factor damp / D_nb folded into the coefficient
                        cf[o] = cf[o] * (ok ? dinv[p + oz * sz + oy * sy + ox] : czero<T>());
                    }
                }
#pragma unroll 1
        for (int r = rlo; r < rhi; ++r) {
            const cplx<T>* __restrict__ src = (MODE == 4 || MODE == 5) ? f + r * vf : u + r * vu;
            cplx<T> xu = czero<T>();
#pragma unroll
            for (int oz = -WZ; oz <= WZ; ++oz)
#pragma unroll
                for (int oy = -WY; oy <= WY; ++oy)
#pragma unroll
                    for (int ox = -WX; ox <= WX; ++ox) {
                        const int o = ((oz + WZ) * NY + (oy + WY)) * NX + (ox + WX);
                        const int64_t q = ((okmask >> o) & 1u) ? p + oz * sz + oy * sy + ox : p;
                        xu = xu + cf[o] * src[q];
                    }
            const cplx<T> fp = f[r * vf + p];
            if (MODE == 1) out[r * vo + p] = src[p] + sc * (fp - xu);
            else if (MODE == 2) out[r * vo + p] = fp - xu;
            else if (MODE == 3) out[r * vo + p] = xu;
            else if (MODE == 4) {
                out[r * vo + p] = sc * fp;
                a.out2[slot][r * a.vo2[slot] + p] = fp - xu;
            } else {
                out[r * vo + p] = sc * fp + sc * (fp - xu);
            }
        }
        return;
    }
    for (int r = rlo; r < rhi; ++r) {
        const cplx<T>* __restrict__ ur = u + r * vu;
        const cplx<T>* __restrict__ fr = f + r * vf;
        cplx<T> xu = czero<T>();
#pragma unroll
        for (int oz = -WZ; oz <= WZ; ++oz) {
            if (k + oz < 0 || k + oz >= d.g[2]) continue;
#pragma unroll
            for (int oy = -WY; oy <= WY; ++oy) {
                if (j + oy < 0 || j + oy >= d.g[1]) continue;
#pragma unroll
                for (int ox = -WX; ox <= WX; ++ox) {
                    if (i + ox < 0 || i + ox >= d.g[0]) continue;
                    const int o = ((oz + WZ) * NY + (oy + WY)) * NX + (ox + WX);
                    const int64_t q = p + oz * sz + oy * sy + ox;
                    cplx<T> v;
                    if (MODE == 4 || MODE == 5) v = dinv[q] * fr[q];
                    else v = ur[q];
                    xu = xu + stencil_coef<T, NST, HALF>(coef, np, o, p, q) * v;
                }
            }
        }
        if (MODE == 1) {
            out[r * vo + p] = ur[p] + sc * (fr[p] - xu);
        } else if (MODE == 2) {
            out[r * vo + p] = fr[p] - xu;
        } else if (MODE == 3) {
            out[r * vo + p] = xu;
        } else if (MODE == 4) {
            out[r * vo + p] = sc * fr[p];
            a.out2[slot][r * a.vo2[slot] + p] = fr[p] - xu;
        } else {
            out[r * vo + p] = sc * fr[p] + sc * (fr[p] - xu);
        }
    }
}

// MIXED is a template parameter so that the 3x3(x3) mixed-intergrid
// kernels are not sized for the wide full-weighting stencils of 3D.
template <class T, int DIM, int MODE, bool MIXED>
__global__ void __launch_bounds__(256)
k_gstencil(GArgs<T> a, int nrhs, int rch) {
    EH_GROUP_POINT(a, d, rch)
    const int kind = a.kind[slot];
    // with full weighting, kinds below DIM are the symmetric, half-stored
    // shear blocks (the mixed restriction is not P^T / 2^d: stored in full)
    if (MIXED) {
        stencil_body<T, 1, 1, (DIM == 3 ? 1 : 0), MODE, false>(a, slot, d, i, j, k, p, sy, sz, rlo, rhi);
        return;
    }
    if (DIM == 2) {
        if (kind == 0) stencil_body<T, 1, 2, 0, MODE, true>(a, slot, d, i, j, k, p, sy, sz, rlo, rhi);
        else if (kind == 1) stencil_body<T, 2, 1, 0, MODE, true>(a, slot, d, i, j, k, p, sy, sz, rlo, rhi);
        else stencil_body<T, 2, 2, 0, MODE, false>(a, slot, d, i, j, k, p, sy, sz, rlo, rhi);
    } else {
        if (kind == 0) stencil_body<T, 1, 2, 2, MODE, true>(a, slot, d, i, j, k, p, sy, sz, rlo, rhi);
        else if (kind == 1) stencil_body<T, 2, 1, 2, MODE, true>(a, slot, d, i, j, k, p, sy, sz, rlo, rhi);
        else if (kind == 2) stencil_body<T, 2, 2, 1, MODE, true>(a, slot, d, i, j, k, p, sy, sz, rlo, rhi);
        else stencil_body<T, 2, 2, 2, MODE, false>(a, slot, d, i, j, k, p, sy, sz, rlo, rhi);
    }
}

// ---------------------------------------------------------------------------
// transfers: restriction (grid = coarse level, reads f as the fine residual,
// writes out on the coarse grid) and prolongation (grid = fine level, adds P
// of f (coarse) into out)

template <class T, int DIM, int NM, bool MIXED>
__device__ __forceinline__ void restrict_body(const GArgs<T>& a, int slot, const Dims& dc, int i, int j, int k,
                                              int64_t p, int rlo, int rhi) {
    using RX = R1<(NM & 1) != 0, MIXED>;
    using RY = R1<(NM & 2) != 0, MIXED>;
    using RZ = R1<(NM & 4) != 0, MIXED>;
    constexpr int SZ = DIM == 3 ? RZ::S : 1;
    const Dims df = a.dc[slot];      // for restriction dc[] holds the FINE grid
    const int64_t fsy = df.g[0], fsz = (int64_t)df.g[0] * df.g[1];
    const int x0 = 2 * i + RX::FIRST, y0 = 2 * j + RY::FIRST, z0 = DIM == 3 ? 2 * k + RZ::FIRST : 0;
    const cplx<T>* r = a.f[slot];
    cplx<T>* fc = a.out[slot];
    const int64_t vsf = a.vf[slot], vsc = a.vo[slot];
    for (int rr = rlo; rr < rhi; ++rr) {
        const cplx<T>* rf = r + rr * vsf;
        cplx<T> s = czero<T>();
#pragma unroll
        for (int aa = 0; aa < SZ; ++aa) {
            const int z = z0 + aa;
            if (DIM == 3 && (z < 0 || z >= df.g[2])) continue;
            const T wz = DIM == 3 ? T(RZ::w(aa)) : T(1);
#pragma unroll
            for (int b = 0; b < RY::S; ++b) {
                const int y = y0 + b;
                if (y < 0 || y >= df.g[1]) continue;
                const T wzy = wz * T(RY::w(b));
                const int64_t row = z * fsz + y * fsy;
#pragma unroll
                for (int cc = 0; cc < RX::S; ++cc) {
                    const int x = x0 + cc;
                    if (x < 0 || x >= df.g[0]) continue;
                    s = s + (wzy * T(RX::w(cc))) * rf[row + x];
                }
            }
        }
        fc[rr * vsc + p] = s;
    }
}

template <class T, int DIM, int NM>
__device__ __forceinline__ void prolong_body(const GArgs<T>& a, int slot, const Dims& df, int i, int j, int k,
                                             int64_t p, int rlo, int rhi) {
    const Dims dc = a.dc[slot];
    int xi[2], yi[2], zi[2];
    float xw[2], yw[2], zw[2];
    p1<(NM & 1) != 0>(i, dc.g[0], xi[0], xi[1], xw[0], xw[1]);
    p1<(NM & 2) != 0>(j, dc.g[1], yi[0], yi[1], yw[0], yw[1]);
    if (DIM == 3) p1<(NM & 4) != 0>(k, dc.g[2], zi[0], zi[1], zw[0], zw[1]);
    else { zi[0] = zi[1] = 0; zw[0] = 1.0f; zw[1] = 0.0f; }
    const int64_t csy = dc.g[0], csz = (int64_t)dc.g[0] * dc.g[1];
    const cplx<T>* ec = a.f[slot];
    cplx<T>* u = a.out[slot];
    const int64_t vsc = a.vf[slot], vsf = a.vo[slot];
    for (int rr = rlo; rr < rhi; ++rr) {
        const cplx<T>* e = ec + rr * vsc;
        cplx<T> s = czero<T>();
#pragma unroll
        for (int aa = 0; aa < (DIM == 3 ? 2 : 1); ++aa)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const T wzy = T(zw[aa]) * T(yw[b]);
                const int64_t row = zi[aa] * csz + yi[b] * csy;
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) s = s + (wzy * T(xw[cc])) * e[row + xi[cc]];
            }
        u[rr * vsf + p] = u[rr * vsf + p] + s;
    }
}

template <class T, int DIM, bool RESTRICT>
__global__ void __launch_bounds__(256)
k_gtransfer(GArgs<T> a, int nrhs, int rch) {
    EH_GROUP_POINT(a, d, rch)
    const int kind = a.kind[slot];
#define EH_TB(NM)                                                                       \
    if (RESTRICT) {                                                                     \
        if (a.mixed) restrict_body<T, DIM, NM, true>(a, slot, d, i, j, k, p, rlo, rhi);     \
        else restrict_body<T, DIM, NM, false>(a, slot, d, i, j, k, p, rlo, rhi);            \
    } else prolong_body<T, DIM, NM>(a, slot, d, i, j, k, p, rlo, rhi);
    if (kind == DIM) { EH_TB(0) }
    else if (kind == 0) { EH_TB(1) }
    else if (kind == 1) { EH_TB(2) }
    else { EH_TB(4) }
#undef EH_TB
}

// ---------------------------------------------------------------------------
// coarsest level: e = Ainv f per slot (one workgroup per row)

struct DenseArgs {
    int ns;
    int N[GMAX];
    const c128* Ainv[GMAX];
};

template <class T, int RB>
__global__ void __launch_bounds__(256)
k_gdense(DenseArgs da, GArgs<T> a) {
    // one row per workgroup: its 256 threads take the columns 256 apart
    // (four row segments of 4 KB in flight per round), so even one block's
    // ~1000 rows keep 16 wavefronts per compute unit reading the matrix
    const int slot = blockIdx.y;
    if (slot >= da.ns) return;
    const int N = da.N[slot];
    const int row = blockIdx.x;
    if (row >= N) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const c128* A = da.Ainv[slot] + (int64_t)row * N;
    const cplx<T>* f = a.f[slot];
    cplx<T>* e = a.out[slot];
    const int64_t vf = a.vf[slot], ve = a.vo[slot];
    double accr[RB], acci[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) { accr[r] = 0.0; acci[r] = 0.0; }
    constexpr int U = 4;
    int c = threadIdx.x;
    for (; c + 256 * (U - 1) < N; c += 256 * U) {
        c128 av[U];
#pragma unroll
        for (int u = 0; u < U; ++u) av[u] = A[c + 256 * u];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const cplx<T> fv = f[r * vf + c + 256 * u];
                accr[r] += av[u].re * double(fv.re) - av[u].im * double(fv.im);
                acci[r] += av[u].re * double(fv.im) + av[u].im * double(fv.re);
            }
    }
    for (; c < N; c += 256) {
        const c128 av = A[c];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const cplx<T> fv = f[r * vf + c];
            accr[r] += av.re * double(fv.re) - av.im * double(fv.im);
            acci[r] += av.re * double(fv.im) + av.im * double(fv.re);
        }
    }
    // fixed-order reduction: within each wavefront, then over the four
    __shared__ double sr[4][RB], si[4][RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        for (int off = 32; off > 0; off >>= 1) {
            accr[r] += __shfl_xor(accr[r], off, 64);
            acci[r] += __shfl_xor(acci[r], off, 64);
        }
        if (lane == 0) { sr[wave][r] = accr[r]; si[wave][r] = acci[r]; }
    }
    __syncthreads();
    if (threadIdx.x < RB) {
        const int r = threadIdx.x;
        const double re = (sr[0][r] + sr[1][r]) + (sr[2][r] + sr[3][r]);
        const double im = (si[0][r] + si[1][r]) + (si[2][r] + si[3][r]);
        e[r * ve + row] = mk<T>(T(re), T(im));
    }
}

// ---------------------------------------------------------------------------
// coupling g_k = r_k - B_k^T e_p for every shear block (eq. prec); r_k is
// rs[r * rss] times the stored vector when rs is given

struct CoupleArgs {
    int ns;
    int kind[GMAX];
    int maxg2;
    Dims d[GMAX];
    const c128* ru[GMAX];
    void* g[GMAX];
    int64_t vg[GMAX];
    double ih[GMAX];
    const double* rs;        // optional per-RHS scale of ru (stride rss)
    int64_t rss;
};

template <class T>
__global__ void __launch_bounds__(256)
k_gcouple(CoupleArgs a, Dims dc, const cplx<T>* __restrict__ ep, int nrhs, int64_t vr, int64_t ve, int rch) {
    EH_GROUP_POINT(a, d, rch)
    const int kaxis = a.kind[slot];
    int c[3] = {i, j, k};
    const int ck = c[kaxis];
    int64_t chi = -1, clo = -1;
    if (ck < dc.g[kaxis]) chi = ((int64_t)c[2] * dc.g[1] + c[1]) * dc.g[0] + c[0];
    if (ck >= 1) {
        c[kaxis] = ck - 1;
        clo = ((int64_t)c[2] * dc.g[1] + c[1]) * dc.g[0] + c[0];
    }
    const c128* ru = a.ru[slot];
    cplx<T>* g = (cplx<T>*)a.g[slot];
    const double ihk = a.ih[slot];
    const int64_t vg = a.vg[slot];
    for (int r = rlo; r < rhi; ++r) {
        c128 gr = mk(0.0, 0.0);
        if (chi >= 0) gr = gr + ccast<double>(ep[r * ve + chi]);
        if (clo >= 0) gr = gr - ccast<double>(ep[r * ve + clo]);
        const double sr = a.rs ? a.rs[r * a.rss] : 1.0;
        g[r * vg + p] = ccast<T>(sr * ru[r * vr + p] - ihk * gr);
    }
}

}  // namespace eh
