// Block-tridiagonal direct solve of the coarsest multigrid level (FP64).
//
// The paper solves the coarsest grid of every block directly (Section
// 4.4.1, "Multigrid setup").  A coarse stencil of half width w_a along axis
// a couples only points whose index along a differs by at most w_a, so
// cutting the grid into groups of w_a consecutive planes (lines in 2D)
// normal to a makes the operator block tridiagonal:
//     L_I x_{I-1} + D_I x_I + U_I x_{I+1} = f_I.
// Setup (block LU without pivoting between groups):
//     S_0 = D_0,  S_I = D_I - L_I W_{I-1},  W_I = S_I^-1 U_I,
// each S_I inverted by blocked Gauss-Jordan (32 x 32 pivot blocks, partial
// pivoting inside each pivot block).  Stored per group, negated couplings:
//     F_I = [S_I^-1 | -S_I^-1 L_I]   (b_I x (b_I + b_{I-1}), row-major)
//     B_I = -W_I                     (b_I x b_{I+1})
// Solve: forward y_I = S_I^-1 f_I - S_I^-1 L_I y_{I-1} = F_I [f_I; y_{I-1}],
// back x_I = y_I + B_I x_{I+1}.  One launch per group and sweep, the right-
// hand sides of a chunk sharing each matrix row read.
#pragma once

#include "eh_common.h"

namespace eh {

// Partition of one block's coarsest grid into groups of planes normal to
// axis `ax`.  Local index m of group I: plane t = I*gsz + m / P, in-plane
// index q = m % P = c[a1] + g[a1] * c[a2].
struct BTPart {
    Dims d;
    Widths w;
    int ax, a1, a2;
    int gsz;        // planes per group (= w[ax])
    int nb;         // groups
    int P;          // points per plane
    __host__ __device__ int planes(int I) const { return min(gsz, d.g[ax] - I * gsz); }
    __host__ __device__ int bsize(int I) const { return (I < 0 || I >= nb) ? 0 : planes(I) * P; }
    __host__ __device__ void coords(int I, int m, int c[3]) const {
        const int t = I * gsz + m / P, q = m % P;
        c[ax] = t;
        c[a1] = q % d.g[a1];
        c[a2] = q / d.g[a1];
    }
    __host__ __device__ int64_t point(const int c[3]) const {
        return ((int64_t)c[2] * d.g[1] + c[1]) * d.g[0] + c[0];
    }
    __host__ __device__ int group(const int c[3]) const { return c[ax] / gsz; }
    __host__ __device__ int local(const int c[3]) const {
        return (c[ax] - (c[ax] / gsz) * gsz) * P + c[a1] + d.g[a1] * c[a2];
    }
    __host__ __device__ bool inside(const int c[3]) const {
        return c[0] >= 0 && c[0] < d.g[0] && c[1] >= 0 && c[1] < d.g[1] && c[2] >= 0 && c[2] < d.g[2];
    }
    __host__ __device__ int offset_index(int ox, int oy, int oz) const {
        return ((oz + w.w[2]) * (2 * w.w[1] + 1) + (oy + w.w[1])) * (2 * w.w[0] + 1) + (ox + w.w[0]);
    }
};

// ---------------------------------------------------------------------------
// setup

// M = S_I = D_I - L_I W_{I-1} for group I, padded to bp x bp with the
// identity.  st: FP64 stencil [nst][N]; Wp: W_{I-1} stored negated
// (b_{I-1} x b_I, row-major), so the update adds L_I Wp.
__global__ void __launch_bounds__(256)
k_bt_schur(BTPart pt, const c128* __restrict__ st, int I, const c128* __restrict__ Wp, c128* __restrict__ M,
           int bp) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (col >= bp || row >= bp) return;
    const int b = pt.bsize(I);
    c128* out = M + (int64_t)row * bp + col;
    if (row >= b || col >= b) {
        *out = mk(row == col ? 1.0 : 0.0, 0.0);
        return;
    }
    int cr[3], cc[3];
    pt.coords(I, row, cr);
    pt.coords(I, col, cc);
    const int64_t N = pt.d.np();
    const int64_t pr = pt.point(cr);
    c128 v = mk(0.0, 0.0);
    const int ox = cc[0] - cr[0], oy = cc[1] - cr[1], oz = cc[2] - cr[2];
    if (abs(ox) <= pt.w.w[0] && abs(oy) <= pt.w.w[1] && abs(oz) <= pt.w.w[2])
        v = st[(int64_t)pt.offset_index(ox, oy, oz) * N + pr];
    if (I > 0) {
        const int bnext = b;   // columns of Wp
        for (int dz = -pt.w.w[2]; dz <= pt.w.w[2]; ++dz)
        for (int dy = -pt.w.w[1]; dy <= pt.w.w[1]; ++dy)
        for (int dx = -pt.w.w[0]; dx <= pt.w.w[0]; ++dx) {
            int cn[3] = {cr[0] + dx, cr[1] + dy, cr[2] + dz};
            if (!pt.inside(cn) || pt.group(cn) != I - 1) continue;
            const c128 l = st[(int64_t)pt.offset_index(dx, dy, dz) * N + pr];
            v = v + l * Wp[(int64_t)pt.local(cn) * bnext + col];
        }
    }
    *out = v;
}

constexpr int GJB = 32;   // pivot block of the blocked Gauss-Jordan inversion

// Pivot block K of M (bp x bp, in place): A_KK <- A_KK^-1 by Gauss-Jordan
// with partial pivoting on [A_KK | I] in LDS.  A zero pivot sets *bad.
__global__ void __launch_bounds__(256)
k_gj_diag(c128* __restrict__ M, int bp, int K, int* __restrict__ bad) {
    __shared__ c128 A[GJB][2 * GJB];
    __shared__ c128 mult[GJB];
    __shared__ int piv;
    const int tid = threadIdx.x;
    const int k0 = K * GJB;
    for (int e = tid; e < GJB * 2 * GJB; e += 256) {
        const int i = e / (2 * GJB), j = e % (2 * GJB);
        A[i][j] = j < GJB ? M[(int64_t)(k0 + i) * bp + k0 + j] : mk(j - GJB == i ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int k = 0; k < GJB; ++k) {
        if (tid == 0) {
            int p = k;
            double best = cabs2(A[k][k]);
            for (int i = k + 1; i < GJB; ++i) {
                const double a = cabs2(A[i][k]);
                if (a > best) { best = a; p = i; }
            }
            if (!(best > 0.0)) { *bad = 1; p = -1; }
            piv = p;
        }
        __syncthreads();
        const int p = piv;
        if (p < 0) return;   // uniform: every thread read the same flag
        if (p != k && tid < 2 * GJB) {
            const c128 t = A[k][tid];
            A[k][tid] = A[p][tid];
            A[p][tid] = t;
        }
        __syncthreads();
        const c128 inv = cdiv(mk(1.0, 0.0), A[k][k]);
        __syncthreads();
        if (tid < 2 * GJB) A[k][tid] = inv * A[k][tid];
        if (tid < GJB) mult[tid] = tid == k ? mk(0.0, 0.0) : A[tid][k];
        __syncthreads();
        for (int e = tid; e < GJB * 2 * GJB; e += 256) {
            const int i = e / (2 * GJB), j = e % (2 * GJB);
            if (i != k) A[i][j] = A[i][j] - mult[i] * A[k][j];
        }
        __syncthreads();
    }
    for (int e = tid; e < GJB * GJB; e += 256) {
        const int i = e / GJB, j = e % GJB;
        M[(int64_t)(k0 + i) * bp + k0 + j] = A[i][GJB + j];
    }
}

// Row panel of pivot block K: A_Kj <- A_KK^-1 A_Kj for every column j
// outside the block (64 columns per workgroup).
__global__ void __launch_bounds__(256)
k_gj_rowpanel(c128* __restrict__ M, int bp, int K) {
    __shared__ c128 Dv[GJB][GJB];
    __shared__ c128 Pn[GJB][64];
    const int tid = threadIdx.x;
    const int k0 = K * GJB, j0 = blockIdx.x * 64;
    for (int e = tid; e < GJB * GJB; e += 256) Dv[e / GJB][e % GJB] = M[(int64_t)(k0 + e / GJB) * bp + k0 + e % GJB];
    for (int e = tid; e < GJB * 64; e += 256) {
        const int i = e / 64, j = j0 + e % 64;
        Pn[i][e % 64] = j < bp ? M[(int64_t)(k0 + i) * bp + j] : mk(0.0, 0.0);
    }
    __syncthreads();
    for (int e = tid; e < GJB * 64; e += 256) {
        const int i = e / 64, jl = e % 64, j = j0 + jl;
        if (j >= bp || (j >= k0 && j < k0 + GJB)) continue;
        c128 acc = mk(0.0, 0.0);
#pragma unroll 8
        for (int m = 0; m < GJB; ++m) acc = acc + Dv[i][m] * Pn[m][jl];
        M[(int64_t)(k0 + i) * bp + j] = acc;
    }
}

// Rank-32 update: A_ij <- A_ij - A_iK A_Kj for i, j outside block K (A_Kj
// already multiplied by A_KK^-1).  64 x 64 output tile per workgroup, each
// thread 4 x 4 entries 16 apart.
__global__ void __launch_bounds__(256)
k_gj_update(c128* __restrict__ M, int bp, int K) {
    __shared__ c128 Ac[64][GJB + 1];
    __shared__ c128 Br[GJB][64];
    const int tid = threadIdx.x;
    const int k0 = K * GJB, i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    for (int e = tid; e < 64 * GJB; e += 256) {
        const int i = e / GJB, m = e % GJB;
        Ac[i][m] = i0 + i < bp ? M[(int64_t)(i0 + i) * bp + k0 + m] : mk(0.0, 0.0);
    }
    for (int e = tid; e < GJB * 64; e += 256) {
        const int m = e / 64, j = e % 64;
        Br[m][j] = j0 + j < bp ? M[(int64_t)(k0 + m) * bp + j0 + j] : mk(0.0, 0.0);
    }
    __syncthreads();
    const int tx = tid % 16, ty = tid / 16;
    double ar[4][4], ai[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) { ar[a][b] = 0.0; ai[a][b] = 0.0; }
    for (int m = 0; m < GJB; ++m) {
        c128 x[4], y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = Ac[ty + 16 * a][m];
#pragma unroll
        for (int b = 0; b < 4; ++b) y[b] = Br[m][tx + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                ar[a][b] += x[a].re * y[b].re - x[a].im * y[b].im;
                ai[a][b] += x[a].re * y[b].im + x[a].im * y[b].re;
            }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + ty + 16 * a;
        if (i >= bp || (i >= k0 && i < k0 + GJB)) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = j0 + tx + 16 * b;
            if (j >= bp || (j >= k0 && j < k0 + GJB)) continue;
            c128* p = M + (int64_t)i * bp + j;
            *p = *p - mk(ar[a][b], ai[a][b]);
        }
    }
}

// Column panel of pivot block K: A_iK <- -A_iK A_KK^-1 for every row i
// outside the block (64 rows per workgroup).
__global__ void __launch_bounds__(256)
k_gj_colpanel(c128* __restrict__ M, int bp, int K) {
    __shared__ c128 Dv[GJB][GJB];
    __shared__ c128 Pn[64][GJB + 1];
    const int tid = threadIdx.x;
    const int k0 = K * GJB, i0 = blockIdx.x * 64;
    for (int e = tid; e < GJB * GJB; e += 256) Dv[e / GJB][e % GJB] = M[(int64_t)(k0 + e / GJB) * bp + k0 + e % GJB];
    for (int e = tid; e < 64 * GJB; e += 256) {
        const int i = e / GJB, m = e % GJB;
        Pn[i][m] = i0 + i < bp ? M[(int64_t)(i0 + i) * bp + k0 + m] : mk(0.0, 0.0);
    }
    __syncthreads();
    for (int e = tid; e < 64 * GJB; e += 256) {
        const int il = e / GJB, k = e % GJB, i = i0 + il;
        if (i >= bp || (i >= k0 && i < k0 + GJB)) continue;
        c128 acc = mk(0.0, 0.0);
#pragma unroll 8
        for (int m = 0; m < GJB; ++m) acc = acc + Pn[il][m] * Dv[m][k];
        M[(int64_t)i * bp + k0 + k] = mk(-acc.re, -acc.im);
    }
}

// Copy S_I^-1 (the leading b x b of M, row stride bp) into the first b
// columns of F_I (row stride ld).
__global__ void __launch_bounds__(256)
k_bt_store_inv(const c128* __restrict__ M, int bp, int b, c128* __restrict__ F, int ld) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (col >= b || row >= b) return;
    F[(int64_t)row * ld + col] = M[(int64_t)row * bp + col];
}

// out[i][j] = -sum_r S_I^-1[i][r] X[r][j] for j in group J = I + dir, X =
// L_I (dir -1) or U_I (dir +1): X[r][j] is the coefficient of point j in
// row r, so r = j - o for each stencil offset o that lands in group I.
// M holds S_I^-1 (row stride bp); out has row stride ld.
__global__ void __launch_bounds__(256)
k_bt_couple(BTPart pt, const c128* __restrict__ st, int I, int dir, const c128* __restrict__ M, int bp,
            c128* __restrict__ out, int ld) {
    const int J = I + dir;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int bJ = pt.bsize(J), bI = pt.bsize(I);
    if (j >= bJ || i >= bI) return;
    int cj[3];
    pt.coords(J, j, cj);
    const int64_t N = pt.d.np();
    const c128* Si = M + (int64_t)i * bp;
    c128 acc = mk(0.0, 0.0);
    for (int oz = -pt.w.w[2]; oz <= pt.w.w[2]; ++oz)
    for (int oy = -pt.w.w[1]; oy <= pt.w.w[1]; ++oy)
    for (int ox = -pt.w.w[0]; ox <= pt.w.w[0]; ++ox) {
        int cr[3] = {cj[0] - ox, cj[1] - oy, cj[2] - oz};
        if (!pt.inside(cr) || pt.group(cr) != I) continue;
        const int64_t pr = pt.point(cr);
        acc = acc + Si[pt.local(cr)] * st[(int64_t)pt.offset_index(ox, oy, oz) * N + pr];
    }
    out[(int64_t)i * ld + j] = mk(-acc.re, -acc.im);
}

// y = X x with an FP64 stencil (the setup's accuracy check).
__global__ void __launch_bounds__(256)
k_stencil_f64(Dims d, Widths w, const c128* __restrict__ st, const c128* __restrict__ x, c128* __restrict__ y) {
    const int64_t N = d.np();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int i = (int)(q % d.g[0]);
    const int j = (int)((q / d.g[0]) % d.g[1]);
    const int k = (int)(q / ((int64_t)d.g[0] * d.g[1]));
    const int NX = 2 * w.w[0] + 1, NY = 2 * w.w[1] + 1;
    c128 acc = mk(0.0, 0.0);
    for (int oz = -w.w[2]; oz <= w.w[2]; ++oz)
    for (int oy = -w.w[1]; oy <= w.w[1]; ++oy)
    for (int ox = -w.w[0]; ox <= w.w[0]; ++ox) {
        const int a = i + ox, b = j + oy, c = k + oz;
        if (a < 0 || a >= d.g[0] || b < 0 || b >= d.g[1] || c < 0 || c >= d.g[2]) continue;
        const int o = ((oz + w.w[2]) * NY + (oy + w.w[1])) * NX + (ox + w.w[0]);
        acc = acc + st[(int64_t)o * N + q] * x[((int64_t)c * d.g[1] + b) * d.g[0] + a];
    }
    y[q] = acc;
}

// ---------------------------------------------------------------------------
// solve

constexpr int BT_MAXS = 4;

// Block-tridiagonal solve of X x = f over the groups I of a partition,
// with S_I the Schur complements, L_I / U_I the couplings to groups I - 1 /
// I + 1, F_I = [S_I^-1 | -S_I^-1 L_I] and B_I = -S_I^-1 U_I:
//   forward  y_I = S_I^-1 f_I + (-S_I^-1 L_I) y_{I-1}
//   back     x_I = y_I + B_I x_{I+1}.
// The first term of the forward sweep does not depend on the sweep, so one
// launch computes it for every group (k_bt_fpart); the sweeps then add, one
// group step per launch, a matrix-vector product with the neighbour
// group's vector in place (k_bt_chain).  Products and sums in FP64.

// Both are matrix-vector products whose vector a group of rows shares: one
// row per wavefront, four per workgroup.  Per chunk of columns each
// wavefront first issues all loads of its row's entries, the workgroup
// stages the vector's chunk (every right-hand side, FP64) in LDS, and each
// lane sums its columns in a fixed order; a butterfly over the wavefront's
// lanes completes the row.  The arithmetic of a right-hand side does not
// depend on the others in the chunk.
// columns per lane and chunk (the staged chunk holds 40 KB at most)
template <int RB>
constexpr int bt_na() { return RB >= 8 ? 5 : 10; }
constexpr int BT_RW = 4;                // rows per workgroup, one per wavefront

template <int RB>
__device__ __forceinline__ void bt_wave_sum(double (&ar)[RB], double (&ai)[RB]) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
        for (int off = 32; off > 0; off >>= 1) {
            ar[r] += __shfl_xor(ar[r], off, 64);
            ai[r] += __shfl_xor(ai[r], off, 64);
        }
}

// Accumulate this wavefront's row A (nc entries; null: no row) times the
// staged vectors, chunk by chunk; stage(c0, w, xs) writes columns c0 ..
// c0 + w - 1 of every right-hand side into xs[r * CW + cc], CW = 64 NA.
template <int RB, class Stage>
__device__ __forceinline__ void bt_rows(const c128* __restrict__ A, int nc, c128* xs, Stage stage,
                                        double (&ar)[RB], double (&ai)[RB]) {
    constexpr int NA = bt_na<RB>(), CW = 64 * NA;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < RB; ++r) { ar[r] = 0.0; ai[r] = 0.0; }
    for (int c0 = 0; c0 < nc; c0 += CW) {
        const int w = min(CW, nc - c0);
        c128 mv[NA];
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int c = lane + 64 * u;
            mv[u] = (A && c < w) ? A[c0 + c] : mk(0.0, 0.0);
        }
        stage(c0, w, xs);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int c = lane + 64 * u;
            if (c < w) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const c128 x = xs[r * CW + c];
                    ar[r] += mv[u].re * x.re - mv[u].im * x.im;
                    ai[r] += mv[u].re * x.im + mv[u].im * x.re;
                }
            }
        }
        if (c0 + CW < nc) __syncthreads();   // the next chunk reuses xs
    }
    bt_wave_sum<RB>(ar, ai);
}

// Every group's S_I^-1 f_I.  Per slot: N points, groups of b0 rows (the
// last may be shorter), nb groups, F_I at mats + offF[I] with rows of b_I +
// b_{I-1} entries, the point permutation in group order, the FP64 work
// vector y (stride N per right-hand side) and f in the level's layout.
template <class T>
struct BTAll {
    int ns;
    int nrhs;
    int N[BT_MAXS], b0[BT_MAXS], nb[BT_MAXS];
    const c128* mats[BT_MAXS];
    const int64_t* offF[BT_MAXS];   // device array, one entry per group
    const int* perm[BT_MAXS];
    c128* y[BT_MAXS];
    const cplx<T>* f[BT_MAXS];
    int64_t vf[BT_MAXS];
};

// Grid (row blocks of BT_RW of the largest group, groups x slots (slot
// fastest), chunks of RB right-hand sides).
template <class T, int RB>
__global__ void __launch_bounds__(256)
k_bt_fpart(BTAll<T> a) {
    constexpr int CW = 64 * bt_na<RB>();
    __shared__ c128 xs[RB * CW];
    const int s = blockIdx.y % a.ns, I = blockIdx.y / a.ns;
    if (I >= a.nb[s]) return;
    const int N = a.N[s], b0 = a.b0[s];
    const int b = min(b0, N - I * b0), bprev = I > 0 ? b0 : 0;
    const int row0 = blockIdx.x * BT_RW;
    if (row0 >= b) return;
    const int row = row0 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const c128* A = row < b ? a.mats[s] + a.offF[s][I] + (int64_t)row * (b + bprev) : nullptr;
    const int* perm = a.perm[s] + (int64_t)I * b0;
    const int r0 = blockIdx.z * RB;
    const int cnt = min(RB, a.nrhs - r0);
    const int64_t vf = a.vf[s];
    const cplx<T>* f = a.f[s] + (int64_t)r0 * vf;
    auto stage = [&](int c0, int w, c128* x) {
        constexpr int K = (CW + 255) / 256;
        int pc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int cc = threadIdx.x + 256 * k;
            pc[k] = cc < w ? perm[c0 + cc] : 0;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int cc = threadIdx.x + 256 * k;
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (cc < w) {
                    const cplx<T> v = r < cnt ? f[r * vf + pc[k]] : czero<T>();
                    x[r * CW + cc] = mk(double(v.re), double(v.im));
                }
        }
    };
    double ar[RB], ai[RB];
    bt_rows<RB>(A, b, xs, stage, ar, ai);
    if (row < b) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (lane == r && r < cnt) a.y[s][(int64_t)(r0 + r) * N + (int64_t)I * b0 + row] = mk(ar[r], ai[r]);
    }
}

// One group step of a sweep for up to BT_MAXS blocks.  Per slot: the rows b
// of the group's matrix (the coupling columns -S_I^-1 L_I of F_I, or B_I),
// its row stride lda, the columns bo (the neighbour group's size), the
// group's entries of the point permutation, the work vector at this group
// (y) and at the neighbour group (yo), stride ldy per right-hand side, and
// (back sweep) the level's vector e in the multigrid precision.
template <class T>
struct BTStep {
    int ns;
    int nrhs;
    const c128* mat[BT_MAXS];
    int b[BT_MAXS], bo[BT_MAXS], lda[BT_MAXS];
    const int* perm[BT_MAXS];
    c128* y[BT_MAXS];
    const c128* yo[BT_MAXS];
    int64_t ldy[BT_MAXS];
    cplx<T>* e[BT_MAXS];
    int64_t ve[BT_MAXS];
};

// y_I += M yo, in place; the back sweep also writes e = x_I in the level's
// layout and precision.  Grid (row blocks of BT_RW, slots, chunks of RB
// right-hand sides).
template <class T, int RB, bool BACK>
__global__ void __launch_bounds__(256)
k_bt_chain(BTStep<T> a) {
    constexpr int CW = 64 * bt_na<RB>();
    __shared__ c128 xs[RB * CW];
    const int s = blockIdx.y;
    if (s >= a.ns) return;
    const int b = a.b[s], bo = a.bo[s];
    const int row0 = blockIdx.x * BT_RW;
    if (row0 >= b) return;
    const int row = row0 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r0 = blockIdx.z * RB;
    const int cnt = min(RB, a.nrhs - r0);
    const int64_t ldy = a.ldy[s];
    // this lane's entry of y (lane r: right-hand side r0 + r), loaded early
    const bool wr = row < b && lane < cnt;
    c128* yp = a.y[s] + (wr ? (int64_t)(r0 + lane) * ldy + row : 0);
    const c128 yv = wr ? *yp : mk(0.0, 0.0);
    const c128* A = row < b ? a.mat[s] + (int64_t)row * a.lda[s] : nullptr;
    const c128* xo = a.yo[s] + (int64_t)r0 * ldy;
    auto stage = [&](int c0, int w, c128* x) {
        constexpr int K = (CW + 255) / 256;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int cc = threadIdx.x + 256 * k;
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (cc < w) x[r * CW + cc] = r < cnt ? xo[r * ldy + c0 + cc] : mk(0.0, 0.0);
        }
    };
    double ar[RB], ai[RB];
    bt_rows<RB>(A, bo, xs, stage, ar, ai);
    if (!wr) return;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (lane == r) { sr = ar[r]; si = ai[r]; }
    const c128 x = mk(yv.re + sr, yv.im + si);
    *yp = x;
    if (BACK) a.e[s][(int64_t)(r0 + lane) * a.ve[s] + a.perm[s][row]] = mk<T>(T(x.re), T(x.im));
}

}  // namespace eh
