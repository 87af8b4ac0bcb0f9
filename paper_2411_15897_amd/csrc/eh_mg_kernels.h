// Multigrid kernels for one acoustic block (Section 4.4.1 of the paper):
// damped Jacobi on the fine (matrix-free) and coarse (stored Galerkin
// stencil) levels, residuals, full-weighting restriction (eqs. Ru1, Rp),
// (bi/tri)linear prolongation, and the dense FP64 coarsest solve.
//
// Launch shape: blockDim (64, 4, 1) -- one wavefront per 64 consecutive x
// points of a row, so every load of a field is a coalesced row segment --
// and gridDim (ceil(gx/64), ceil(gy/4), gz).  Vectors of several
// right-hand sides are stored one after the other with stride `vs`.
#pragma once

#include "eh_common.h"

namespace eh {

#define EH_POINT_INDEX(d)                                              \
    const int i = blockIdx.x * blockDim.x + threadIdx.x;               \
    const int j = blockIdx.y * blockDim.y + threadIdx.y;               \
    const int k = blockIdx.z;                                          \
    if (i >= (d).g[0] || j >= (d).g[1]) return;                        \
    const int64_t sx = 1, sy = (d).g[0], sz = (int64_t)(d).g[0] * (d).g[1]; \
    const int64_t p = k * sz + j * sy + i;                             \
    (void)sx;

// Off-diagonal couplings of a fine-level acoustic block at one point.
// The operator is X u = D u - sum_nb c_nb u_nb with real c_nb.
//  KIND 0 (A_k): symmetric edge weights; wa[p] couples p and p + e_a
//                (zero on the last point along a).
//  KIND 1 (H_p): X = B B^T diag(w) - mass: the coupling from p to a
//                neighbour nb along a is w[nb] / h_a^2.
template <class T, int KIND, int DIM>
struct FineCoef {
    T cp[3], cm[3];
    __device__ __forceinline__ void load(const Dims& d, int i, int j, int k, int64_t p,
                                         const T* __restrict__ w0, const T* __restrict__ w1,
                                         const T* __restrict__ w2, T ih0, T ih1, T ih2) {
        const int64_t sy = d.g[0], sz = (int64_t)d.g[0] * d.g[1];
        if (KIND == 0) {
            cp[0] = (i + 1 < d.g[0]) ? w0[p] : T(0);
            cm[0] = (i > 0) ? w0[p - 1] : T(0);
            cp[1] = (j + 1 < d.g[1]) ? w1[p] : T(0);
            cm[1] = (j > 0) ? w1[p - sy] : T(0);
            if (DIM == 3) {
                cp[2] = (k + 1 < d.g[2]) ? w2[p] : T(0);
                cm[2] = (k > 0) ? w2[p - sz] : T(0);
            }
        } else {
            cp[0] = (i + 1 < d.g[0]) ? w0[p + 1] * ih0 : T(0);
            cm[0] = (i > 0) ? w0[p - 1] * ih0 : T(0);
            cp[1] = (j + 1 < d.g[1]) ? w0[p + sy] * ih1 : T(0);
            cm[1] = (j > 0) ? w0[p - sy] * ih1 : T(0);
            if (DIM == 3) {
                cp[2] = (k + 1 < d.g[2]) ? w0[p + sz] * ih2 : T(0);
                cm[2] = (k > 0) ? w0[p - sz] * ih2 : T(0);
            }
        }
    }
    // sum_nb c_nb u_nb
    __device__ __forceinline__ cplx<T> offsum(const Dims& d, int i, int j, int k, int64_t p,
                                              const cplx<T>* __restrict__ u) const {
        const int64_t sy = d.g[0], sz = (int64_t)d.g[0] * d.g[1];
        cplx<T> s = czero<T>();
        if (i + 1 < d.g[0]) s = s + cp[0] * u[p + 1];
        if (i > 0) s = s + cm[0] * u[p - 1];
        if (j + 1 < d.g[1]) s = s + cp[1] * u[p + sy];
        if (j > 0) s = s + cm[1] * u[p - sy];
        if (DIM == 3) {
            if (k + 1 < d.g[2]) s = s + cp[2] * u[p + sz];
            if (k > 0) s = s + cm[2] * u[p - sz];
        }
        return s;
    }
};

// mode 0: out = damp D^-1 f                         (first sweep, zero guess)
// mode 1: out = u + damp D^-1 (f - X u)             (Jacobi sweep)
// mode 2: out = f - X u                             (residual)
// mode 3: out = X u                                 (operator apply)
// Strides between right-hand sides: vf (f), vu (u), vo (out).
template <class T, int KIND, int DIM, int MODE>
__global__ void __launch_bounds__(256)
k_fine(Dims d, const T* __restrict__ w0, const T* __restrict__ w1, const T* __restrict__ w2,
       T ih0, T ih1, T ih2, const cplx<T>* __restrict__ D, const cplx<T>* __restrict__ f,
       const cplx<T>* __restrict__ u, cplx<T>* __restrict__ out, T damp, int nrhs,
       int64_t vf, int64_t vu, int64_t vo) {
    EH_POINT_INDEX(d)
    const cplx<T> Dp = D[p];
    if (MODE == 0) {
        const cplx<T> sc = cdiv(mk<T>(damp, T(0)), Dp);
        for (int r = 0; r < nrhs; ++r) out[r * vo + p] = sc * f[r * vf + p];
        return;
    }
    FineCoef<T, KIND, DIM> c;
    c.load(d, i, j, k, p, w0, w1, w2, ih0, ih1, ih2);
    if (MODE == 1) {
        const cplx<T> sc = cdiv(mk<T>(damp, T(0)), Dp);
        for (int r = 0; r < nrhs; ++r) {
            const cplx<T>* ur = u + r * vu;
            const cplx<T> up = ur[p];
            const cplx<T> res = f[r * vf + p] - Dp * up + c.offsum(d, i, j, k, p, ur);
            out[r * vo + p] = up + sc * res;
        }
    } else if (MODE == 2) {
        for (int r = 0; r < nrhs; ++r) {
            const cplx<T>* ur = u + r * vu;
            out[r * vo + p] = f[r * vf + p] - Dp * ur[p] + c.offsum(d, i, j, k, p, ur);
        }
    } else {
        for (int r = 0; r < nrhs; ++r) {
            const cplx<T>* ur = u + r * vu;
            out[r * vo + p] = Dp * ur[p] - c.offsum(d, i, j, k, p, ur);
        }
    }
}

// Coarse levels: stored Galerkin stencil coef[o * np + p], offsets o over
// (-WX..WX) x (-WY..WY) x (-WZ..WZ), x fastest.  Couplings to points outside
// the grid are zero by construction and are not read.
template <class T, int WX, int WY, int WZ, int MODE>
__global__ void __launch_bounds__(256)
k_stencil(Dims d, const cplx<T>* __restrict__ coef, const cplx<T>* __restrict__ f,
          const cplx<T>* __restrict__ u, cplx<T>* __restrict__ out, T damp, int nrhs,
          int64_t vf, int64_t vu, int64_t vo) {
    EH_POINT_INDEX(d)
    const int64_t np = d.np();
    constexpr int NX = 2 * WX + 1, NY = 2 * WY + 1;
    constexpr int CENTRE = (WZ * NY + WY) * NX + WX;
    const cplx<T> Dp = coef[CENTRE * np + p];
    if (MODE == 0) {
        const cplx<T> sc = cdiv(mk<T>(damp, T(0)), Dp);
        for (int r = 0; r < nrhs; ++r) out[r * vo + p] = sc * f[r * vf + p];
        return;
    }
    for (int r = 0; r < nrhs; ++r) {
        const cplx<T>* ur = u + r * vu;
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
                    xu = xu + coef[o * np + p] * ur[p + oz * sz + oy * sy + ox];
                }
            }
        }
        if (MODE == 1) {
            const cplx<T> sc = cdiv(mk<T>(damp, T(0)), Dp);
            out[r * vo + p] = ur[p] + sc * (f[r * vf + p] - xu);
        } else if (MODE == 2) {
            out[r * vo + p] = f[r * vf + p] - xu;
        } else {
            out[r * vo + p] = xu;
        }
    }
}

// 1D transfer weights.  Nodal axis: coarse node I covers fine nodes
// 2I-1, 2I, 2I+1 with restriction weights 1/4, 1/2, 1/4 (eq. Ru1, nodal
// factor).  Cell-centred axis: coarse cell I covers fine cells 2I-1..2I+2
// with 1/8, 3/8, 3/8, 1/8 (eqs. Ru1, Rp, cell-centred factor).  Fine
// indices outside [0, nf) are dropped.  Restriction R = P^T / 2^d, so the
// prolongation weights are 2x these per axis.
struct Transfer1D {
    int idx[4];
    float wt[4];
    int n;
    __device__ __forceinline__ void restrict_support(int I, bool nodal, int nf) {
        n = 0;
        if (nodal) {
            const int ks[3] = {2 * I - 1, 2 * I, 2 * I + 1};
            const float ws[3] = {0.25f, 0.5f, 0.25f};
            for (int t = 0; t < 3; ++t)
                if (ks[t] >= 0 && ks[t] < nf) { idx[n] = ks[t]; wt[n] = ws[t]; ++n; }
        } else {
            const int ks[4] = {2 * I - 1, 2 * I, 2 * I + 1, 2 * I + 2};
            const float ws[4] = {0.125f, 0.375f, 0.375f, 0.125f};
            for (int t = 0; t < 4; ++t)
                if (ks[t] >= 0 && ks[t] < nf) { idx[n] = ks[t]; wt[n] = ws[t]; ++n; }
        }
    }
    // coarse parents of fine index l with interpolation weights
    __device__ __forceinline__ void prolong_parents(int l, bool nodal, int nc) {
        n = 0;
        if (nodal) {
            if ((l & 1) == 0) { idx[0] = l >> 1; wt[0] = 1.0f; n = 1; }
            else { idx[0] = (l - 1) >> 1; wt[0] = 0.5f; idx[1] = (l + 1) >> 1; wt[1] = 0.5f; n = 2; }
        } else {
            const int I = l >> 1;
            idx[0] = I; wt[0] = 0.75f; n = 1;
            const int nb = (l & 1) ? I + 1 : I - 1;
            if (nb >= 0 && nb < nc) { idx[1] = nb; wt[1] = 0.25f; n = 2; }
        }
    }
};

// fc = R r on the coarse grid
template <class T>
__global__ void __launch_bounds__(256)
k_restrict(Dims df, Dims dc, int nodal_mask, const cplx<T>* __restrict__ r,
           cplx<T>* __restrict__ fc, int nrhs, int64_t vsf, int64_t vsc) {
    EH_POINT_INDEX(dc)
    Transfer1D tx, ty, tz;
    tx.restrict_support(i, nodal_mask & 1, df.g[0]);
    ty.restrict_support(j, nodal_mask & 2, df.g[1]);
    if (df.g[2] > 1 || (nodal_mask & 4)) tz.restrict_support(k, nodal_mask & 4, df.g[2]);
    else { tz.n = 1; tz.idx[0] = 0; tz.wt[0] = 1.0f; }
    const int64_t fsy = df.g[0], fsz = (int64_t)df.g[0] * df.g[1];
    for (int rr = 0; rr < nrhs; ++rr) {
        const cplx<T>* rf = r + rr * vsf;
        cplx<T> s = czero<T>();
        for (int a = 0; a < tz.n; ++a) {
            for (int b = 0; b < ty.n; ++b) {
                const T wzy = T(tz.wt[a]) * T(ty.wt[b]);
                const int64_t base = tz.idx[a] * fsz + ty.idx[b] * fsy;
                for (int c = 0; c < tx.n; ++c) s = s + (wzy * T(tx.wt[c])) * rf[base + tx.idx[c]];
            }
        }
        fc[rr * vsc + p] = s;
    }
}

// u += P ec on the fine grid (P = 2^d R^T: bi/trilinear interpolation)
template <class T>
__global__ void __launch_bounds__(256)
k_prolong_add(Dims df, Dims dc, int nodal_mask, const cplx<T>* __restrict__ ec,
              cplx<T>* __restrict__ u, int nrhs, int64_t vsf, int64_t vsc) {
    EH_POINT_INDEX(df)
    Transfer1D tx, ty, tz;
    tx.prolong_parents(i, nodal_mask & 1, dc.g[0]);
    ty.prolong_parents(j, nodal_mask & 2, dc.g[1]);
    if (df.g[2] > 1 || (nodal_mask & 4)) tz.prolong_parents(k, nodal_mask & 4, dc.g[2]);
    else { tz.n = 1; tz.idx[0] = 0; tz.wt[0] = 1.0f; }
    const int64_t csy = dc.g[0], csz = (int64_t)dc.g[0] * dc.g[1];
    for (int rr = 0; rr < nrhs; ++rr) {
        const cplx<T>* e = ec + rr * vsc;
        cplx<T> s = czero<T>();
        for (int a = 0; a < tz.n; ++a) {
            for (int b = 0; b < ty.n; ++b) {
                const T wzy = T(tz.wt[a]) * T(ty.wt[b]);
                const int64_t base = tz.idx[a] * csz + ty.idx[b] * csy;
                for (int c = 0; c < tx.n; ++c) s = s + (wzy * T(tx.wt[c])) * e[base + tx.idx[c]];
            }
        }
        u[rr * vsf + p] = u[rr * vsf + p] + s;
    }
}

// Coarsest level: e = Ainv f with the dense FP64 inverse (row-major N x N).
// One wavefront per row; lanes stride along the row (coalesced); RB
// right-hand sides share each read of the row.
template <class T, int RB>
__global__ void __launch_bounds__(256)
k_dense_apply(int N, const c128* __restrict__ Ainv, const cplx<T>* __restrict__ f,
              cplx<T>* __restrict__ e, int64_t vf, int64_t ve) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= N) return;
    const c128* a = Ainv + (int64_t)row * N;
    double accr[RB], acci[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) { accr[r] = 0.0; acci[r] = 0.0; }
    for (int c = lane; c < N; c += 64) {
        const c128 av = a[c];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const cplx<T> fv = f[r * vf + c];
            accr[r] += av.re * double(fv.re) - av.im * double(fv.im);
            acci[r] += av.re * double(fv.im) + av.im * double(fv.re);
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        for (int off = 32; off > 0; off >>= 1) {
            accr[r] += __shfl_xor(accr[r], off, 64);
            acci[r] += __shfl_xor(acci[r], off, 64);
        }
        if (lane == 0) e[r * ve + row] = mk<T>(T(accr[r]), T(acci[r]));
    }
}

}  // namespace eh
