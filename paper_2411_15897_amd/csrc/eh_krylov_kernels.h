// FP64 reductions and vector updates of the flexible GMRES Arnoldi process
// (classical Gram-Schmidt applied twice).  Reductions are deterministic:
// every block writes its partial sums, a second kernel adds them in a fixed
// order, so FP64 runs are bitwise repeatable.
//
// Basis layout: vector i of right-hand side r starts at V + (i*nrhs + r)*n.
#pragma once

#include "eh_common.h"

namespace eh {

constexpr int KRY_THREADS = 256;
constexpr int KRY_MAXM = 32;   // columns handled by one pass

// MODE 0: partial[i] = sum_p conj(V_i[p]) w[p]                   (i < m)
// MODE 1: wout <- w - sum_i c_i V_i;  partial[i] = sum conj(V_i) wout   (update + dot)
// MODE 2: wout <- w - sum_i c_i V_i;  partial[0] = sum |wout|^2         (update + norm)
// MODE 3: partial[0] = sum |w|^2
// MODE 4: partial[i] = sum conj(V_i) w and partial[m + i] = sum conj(V_i) V_{m-1}
//         (projections of w and the newest column of the Gram matrix V^H V)
// grid: (nblk, nrhs); block b owns the KRY_E * 256 entries starting at
// b * KRY_E * 256 (each thread KRY_E of them, 256 apart: coalesced).
// partial layout [r][i][blk] (i < m, or 1 for norms); coef layout [r][i].
constexpr int KRY_E = 4;
template <int MODE>
__global__ void __launch_bounds__(KRY_THREADS)
k_gs(int64_t n, int m, int nrhs, const c128* __restrict__ V, const c128* w,
     const c128* __restrict__ coef, c128* __restrict__ partial, c128* wout) {
    __shared__ double lre[4][2 * KRY_MAXM], lim[4][2 * KRY_MAXM];
    const int r = blockIdx.y;
    const int nblk = gridDim.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * (KRY_E * KRY_THREADS) + threadIdx.x;
    const c128* wr = w + (int64_t)r * n;
    c128 wv[KRY_E];
#pragma unroll
    for (int e = 0; e < KRY_E; ++e) {
        const int64_t p = base + e * KRY_THREADS;
        wv[e] = p < n ? wr[p] : mk(0.0, 0.0);
    }
    if (MODE == 1 || MODE == 2) {
        for (int t = 0; t < m; ++t) {
            const c128 cf = coef[r * m + t];
            const c128* Vt = V + ((int64_t)t * nrhs + r) * n;
#pragma unroll
            for (int e = 0; e < KRY_E; ++e) {
                const int64_t p = base + e * KRY_THREADS;
                if (p < n) wv[e] = wv[e] - cf * Vt[p];
            }
        }
        c128* wo = wout + (int64_t)r * n;
#pragma unroll
        for (int e = 0; e < KRY_E; ++e) {
            const int64_t p = base + e * KRY_THREADS;
            if (p < n) wo[p] = wv[e];
        }
    }
    int mm = 1;
    if (MODE == 4) {
        mm = 2 * m;
        c128 vl[KRY_E];
        const c128* Vl = V + ((int64_t)(m - 1) * nrhs + r) * n;
#pragma unroll
        for (int e = 0; e < KRY_E; ++e) {
            const int64_t p = base + e * KRY_THREADS;
            vl[e] = p < n ? Vl[p] : mk(0.0, 0.0);
        }
        for (int t = 0; t < m; ++t) {
            const c128* Vt = V + ((int64_t)t * nrhs + r) * n;
            double ar = 0.0, ai = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
            for (int e = 0; e < KRY_E; ++e) {
                const int64_t p = base + e * KRY_THREADS;
                if (p < n) {
                    const c128 v = t == m - 1 ? vl[e] : Vt[p];   // the newest column is in registers
                    ar += v.re * wv[e].re + v.im * wv[e].im;
                    ai += v.re * wv[e].im - v.im * wv[e].re;
                    gr += v.re * vl[e].re + v.im * vl[e].im;
                    gi += v.re * vl[e].im - v.im * vl[e].re;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                ar += __shfl_xor(ar, off, 64);
                ai += __shfl_xor(ai, off, 64);
                gr += __shfl_xor(gr, off, 64);
                gi += __shfl_xor(gi, off, 64);
            }
            if (lane == 0) {
                lre[wave][t] = ar; lim[wave][t] = ai;
                lre[wave][m + t] = gr; lim[wave][m + t] = gi;
            }
        }
    } else if (MODE == 0 || MODE == 1) {
        mm = m;
        for (int t = 0; t < m; ++t) {
            const c128* Vt = V + ((int64_t)t * nrhs + r) * n;
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int e = 0; e < KRY_E; ++e) {
                const int64_t p = base + e * KRY_THREADS;
                if (p < n) {
                    const c128 v = Vt[p];
                    ar += v.re * wv[e].re + v.im * wv[e].im;
                    ai += v.re * wv[e].im - v.im * wv[e].re;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                ar += __shfl_xor(ar, off, 64);
                ai += __shfl_xor(ai, off, 64);
            }
            if (lane == 0) { lre[wave][t] = ar; lim[wave][t] = ai; }
        }
    } else {
        double a = 0.0;
#pragma unroll
        for (int e = 0; e < KRY_E; ++e) a += wv[e].re * wv[e].re + wv[e].im * wv[e].im;
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        if (lane == 0) { lre[wave][0] = a; lim[wave][0] = 0.0; }
    }
    __syncthreads();
    if (threadIdx.x < mm) {
        const int t = threadIdx.x;
        const double sr = (lre[0][t] + lre[1][t]) + (lre[2][t] + lre[3][t]);
        const double si = (lim[0][t] + lim[1][t]) + (lim[2][t] + lim[3][t]);
        partial[((int64_t)r * mm + t) * nblk + blockIdx.x] = mk(sr, si);
    }
}

// out[r][i] = sum_blk partial[r][i][blk]: one block per (i, r), fixed-order
// tree, so the result does not depend on timing.
__global__ void __launch_bounds__(256)
k_reduce_partials(int nblk, int m, int nrhs, const c128* __restrict__ partial, c128* __restrict__ out) {
    __shared__ double sre[256], sim[256];
    const int i = blockIdx.x, r = blockIdx.y;
    const c128* pr = partial + ((int64_t)r * m + i) * nblk;
    double ar = 0.0, ai = 0.0;
    // eight partials in flight per thread, then the remainder (fixed order)
    constexpr int U = 8;
    int b = threadIdx.x;
    for (; b + (U - 1) * 256 < nblk; b += U * 256) {
        c128 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = pr[b + u * 256];
#pragma unroll
        for (int u = 0; u < U; ++u) { ar += v[u].re; ai += v[u].im; }
    }
    for (; b < nblk; b += 256) {
        const c128 v = pr[b];
        ar += v.re; ai += v.im;
    }
    sre[threadIdx.x] = ar; sim[threadIdx.x] = ai;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sre[threadIdx.x] += sre[threadIdx.x + s];
            sim[threadIdx.x] += sim[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r * m + i] = mk(sre[0], sim[0]);
}

// out = value (graph-safe fill)
template <class V>
__global__ void __launch_bounds__(256)
k_fill(int64_t n, V* __restrict__ out, V value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) out[p] = value;
}

// dst[r * vd + q] = src[r * vs + q] for q < n, r < nrhs (graph-safe copy)
template <class V>
__global__ void __launch_bounds__(256)
k_copy_strided(int64_t n, int nrhs, const V* __restrict__ src, int64_t vs, V* __restrict__ dst, int64_t vd) {
    const int r = blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        dst[(int64_t)r * vd + q] = src[(int64_t)r * vs + q];
}

// out = a - b
__global__ void __launch_bounds__(256)
k_sub(int64_t n, const c128* __restrict__ a, const c128* __restrict__ b, c128* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
        out[p] = a[p] - b[p];
}

// x[r] += sum_{i < jr[r]} y[r][i] Z_i[r]   (Z in the multigrid precision;
// only the jr[r] columns built for that right-hand side in this cycle are
// read -- later columns may hold stale or uninitialised data; y has row
// stride mstride)
template <class T>
__global__ void __launch_bounds__(256)
k_xupdate(int64_t n, const int* __restrict__ jr, int mstride, int nrhs, const cplx<T>* __restrict__ Z,
          const c128* __restrict__ y, c128* __restrict__ x) {
    const int r = blockIdx.y;
    const int mcount = jr[r];
    if (mcount == 0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        c128 s = x[(int64_t)r * n + p];
        for (int i = 0; i < mcount; ++i)
            s = s + y[r * mstride + i] * ccast<double>(Z[((int64_t)i * nrhs + r) * n + p]);
        x[(int64_t)r * n + p] = s;
    }
}

// ---------------------------------------------------------------------------
// Arnoldi bookkeeping on the device
//
// The small per-step arithmetic of flexible GMRES -- the second-pass
// Gram-Schmidt coefficients, the Givens rotations of the new Hessenberg
// column, the residual estimate, the convergence and breakdown tests and the
// triangular solve at the end of a cycle -- runs in the kernels below, so
// Arnoldi steps queue back to back and the host only reads a short status
// record per step (written straight into pinned host memory).
//
// Basis columns are stored unnormalised: the stored column i of RHS r is
// v_i / sv[r][i].  Readers of a column as a vector (the distributor and the
// coupling of the preconditioner) multiply by sv; the Gram-Schmidt
// coefficients fold it in here, so no pass over the vectors is spent on
// normalisation.

struct ArnStatus {
    double est;    // |g_{j+1}| / ||b||, the FGMRES residual estimate
    double rel;    // cycle start only: ||b - H x|| / ||b|| in FP64
    int active;    // still iterating in this cycle
    int its;       // preconditioner applications so far
    int done;      // converged at a cycle start, or a zero right-hand side
    int bad;       // a non-finite value was met
};

struct ArnState {
    int m;           // restart length (layout stride)
    int nrhs;
    double* tol;     // [1]
    double* sv;      // [r][m+1] column scales
    c128* gram;      // [r][m][m] gram[(r*m + q)*m + i] = v_i^H v_q for i <= q
    c128* hcol;      // [r][m] Hessenberg column of the current step
    c128* R;         // [r][m][m+1] rotated Hessenberg columns
    double* cs;      // [r][m] rotation cosines
    c128* sn;        // [r][m] rotation sines
    c128* g;         // [r][m+1] rotated right-hand side beta e_1
    c128* y;         // [r][m] least-squares solution of the cycle
    double* bnorm;   // [r]
    double* est;     // [r]
    int* jr;         // [r] columns built in this cycle
    int* act;        // [r]
    int* its;        // [r]
    int* done;       // [r]
};

// Cycle start.  nrm[r] = |r_0|^2 of the residual held in stored column 0.
// On the first cycle (x = 0) the residual is b itself and fixes ||b||.
__global__ void __launch_bounds__(64)
k_arn_start(ArnState s, const c128* __restrict__ nrm, int first, double tol, ArnStatus* out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0 && first) s.tol[0] = tol;
    if (r >= s.nrhs) return;
    const int m = s.m;
    const double beta = sqrt(fmax(nrm[r].re, 0.0));
    if (first) {
        s.bnorm[r] = beta;
        s.done[r] = beta == 0.0;
        s.est[r] = beta == 0.0 ? 0.0 : 1.0;
        s.its[r] = 0;
    }
    const double bn = s.bnorm[r];
    const double rel = bn > 0.0 ? beta / bn : 0.0;
    if (!s.done[r] && rel < tol) {
        s.done[r] = 1;
        s.est[r] = rel;
    }
    const int act = !s.done[r];
    s.act[r] = act;
    s.jr[r] = 0;
    s.sv[r * (m + 1)] = act ? 1.0 / beta : 0.0;
    for (int q = 0; q <= m; ++q) s.g[r * (m + 1) + q] = mk(q == 0 ? beta : 0.0, 0.0);
    ArnStatus st;
    st.est = s.est[r];
    st.rel = rel;
    st.active = act;
    st.its = s.its[r];
    st.done = s.done[r];
    st.bad = !isfinite(beta);
    out[r] = st;
}

// Second-pass coefficients of step j (CGS2 in two passes).  The first pass
// gave a_i = stored_i^H w and b_i = stored_i^H stored_j (d1 row r:
// [a_0..a_j, b_0..b_j]).  With h1_i = sv_i a_i and the Gram column
// G_ij = sv_i sv_j b_i of the normalised basis, the reorthogonalised column
// is hcol = h1 + V^H (w - V h1) = 2 h1 - G h1, and the update weight on the
// stored column i is coef_i = sv_i hcol_i.  One block per RHS.
__global__ void __launch_bounds__(64)
k_arn_coef(ArnState s, int j, const c128* __restrict__ d1, c128* __restrict__ coef) {
    __shared__ c128 h1[KRY_MAXM], gj[KRY_MAXM];
    const int r = blockIdx.x, i = threadIdx.x, J = j + 1, m = s.m;
    const double* sv = s.sv + r * (m + 1);
    const c128* dr = d1 + (int64_t)r * 2 * J;
    c128* gram = s.gram + (int64_t)r * m * m;
    if (i < J) {
        const double si = sv[i];
        h1[i] = si * dr[i];
        gj[i] = (si * sv[j]) * dr[J + i];
        gram[(int64_t)j * m + i] = gj[i];
    }
    __syncthreads();
    if (i < J) {
        c128 gh = czero<double>();
        for (int q = 0; q < J; ++q) {
            c128 gi;   // G_iq: stored by column q (q >= i) or as conj of column i
            if (q >= i) gi = (q == j) ? gj[i] : gram[(int64_t)q * m + i];
            else gi = (i == j) ? cconj(gj[q]) : cconj(gram[(int64_t)i * m + q]);
            gh = gh + gi * h1[q];
        }
        const c128 hc = 2.0 * h1[i] - gh;
        s.hcol[r * m + i] = hc;
        coef[r * J + i] = s.act[r] ? sv[i] * hc : czero<double>();
    }
}

// Hessenberg column of step j: the earlier rotations, a new rotation that
// zeroes the subdiagonal hn = ||w - V hcol|| (nrm[r] = hn^2), the residual
// estimate, and the convergence / breakdown test.  The new column's scale
// is 1/hn while the RHS stays active, 0 after.  One thread per RHS.
__global__ void __launch_bounds__(64)
k_arn_givens(ArnState s, int j, const c128* __restrict__ nrm, ArnStatus* out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= s.nrhs) return;
    const int m = s.m;
    double* sv = s.sv + r * (m + 1);
    ArnStatus st;
    st.rel = -1.0;
    st.done = s.done[r];
    if (!s.act[r]) {
        sv[j + 1] = 0.0;
        st.est = s.est[r];
        st.active = 0;
        st.its = s.its[r];
        st.bad = 0;
        out[r] = st;
        return;
    }
    const double hn = sqrt(fmax(nrm[r].re, 0.0));
    c128* col = s.R + ((int64_t)r * m + j) * (m + 1);
    double w0 = hn * hn;
    for (int i = 0; i <= j; ++i) {
        col[i] = s.hcol[r * m + i];
        w0 += cabs2(col[i]);
    }
    w0 = sqrt(w0);
    col[j + 1] = mk(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const double ci = s.cs[r * m + i];
        const c128 si = s.sn[r * m + i];
        const c128 a = col[i], b = col[i + 1];
        col[i] = ci * a + si * b;
        col[i + 1] = ci * b - cconj(si) * a;
    }
    const c128 a = col[j];
    const double aa = sqrt(cabs2(a));
    const double nu = sqrt(cabs2(a) + hn * hn);
    double ci;
    c128 si;
    if (aa == 0.0) {
        ci = 0.0;
        si = mk(1.0, 0.0);
    } else {
        ci = aa / nu;
        si = (hn / (nu * aa)) * a;
    }
    s.cs[r * m + j] = ci;
    s.sn[r * m + j] = si;
    col[j] = ci * a + si * col[j + 1];
    col[j + 1] = czero<double>();
    c128* g = s.g + r * (m + 1);
    g[j + 1] = -1.0 * (cconj(si) * g[j]);
    g[j] = ci * g[j];
    s.jr[r] = j + 1;
    const int its = s.its[r] + 1;
    s.its[r] = its;
    const double est = sqrt(cabs2(g[j + 1])) / s.bnorm[r];
    s.est[r] = est;
    const int bad = !isfinite(est);
    const bool brk = hn <= 1e-14 * w0;
    const int act = !(est < s.tol[0] || brk || bad);
    s.act[r] = act;
    sv[j + 1] = act ? 1.0 / hn : 0.0;
    st.est = est;
    st.active = act;
    st.its = its;
    st.bad = bad;
    out[r] = st;
}

// A cycle start that drops finished right-hand sides from the batch: slot i
// takes the state of slot map[i] (map increasing, so map[i] >= i and one
// thread moving the slots in order never overwrites a slot it has still to
// read).  What moves is the state that outlives a cycle (the norm of b, the
// estimate, the counts and flags) and the entries k_arn_start has just
// written for the new cycle (scales, rotated right-hand side).
__global__ void __launch_bounds__(64)
k_arn_compact(ArnState s, const int* __restrict__ map, int k) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int m = s.m;
    for (int i = 0; i < k; ++i) {
        const int q = map[i];
        if (q == i) continue;
        s.bnorm[i] = s.bnorm[q];
        s.est[i] = s.est[q];
        s.its[i] = s.its[q];
        s.done[i] = s.done[q];
        s.act[i] = s.act[q];
        s.jr[i] = s.jr[q];
        for (int t = 0; t <= m; ++t) {
            s.sv[i * (m + 1) + t] = s.sv[q * (m + 1) + t];
            s.g[i * (m + 1) + t] = s.g[q * (m + 1) + t];
        }
    }
}

// End of a cycle: y = R^{-1} g over the jr[r] columns built (back
// substitution on the rotated Hessenberg matrix).  One thread per RHS.
__global__ void __launch_bounds__(64)
k_arn_solve(ArnState s) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= s.nrhs) return;
    const int m = s.m, jj = s.jr[r];
    const c128* R = s.R + (int64_t)r * m * (m + 1);
    c128* y = s.y + r * m;
    for (int i = jj - 1; i >= 0; --i) {
        c128 acc = s.g[r * (m + 1) + i];
        for (int q = i + 1; q < jj; ++q) acc = acc - R[(int64_t)q * (m + 1) + i] * y[q];
        y[i] = cdiv(acc, R[(int64_t)i * (m + 1) + i]);
    }
}

}  // namespace eh
