// Building blocks of the multigrid kernels (Section 4.4.1 of the paper):
// the fine-level matrix-free couplings of an acoustic block and the 1D
// weights of full-weighting restriction (eqs. Ru1, Rp) and (bi/tri)linear
// prolongation.  The kernels themselves are in eh_group_kernels.h.
//
// Launch shape used throughout: blockDim (64, 4, 1) -- one wavefront per 64
// consecutive x points of a row, so every load of a field is a coalesced
// row segment -- and gridDim (ceil(gx/64), ceil(gy/4), gz).
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
//  KIND 2 (H_p built with the Remark's A~_p = B A_f(mu) B^T - w^2 M_p):
//                the coupling across a face depends on the face and the
//                neighbour, (1 + mu_f / (lambda+mu)_nb) / h_a^2; wa holds
//                the pair (to p + e_a, to p - e_a) per point, interleaved.
template <class T, int KIND, int DIM>
struct FineCoef {
    T cp[3], cm[3];
    __device__ __forceinline__ void load(const Dims& d, int i, int j, int k, int64_t p,
                                         const T* __restrict__ w0, const T* __restrict__ w1,
                                         const T* __restrict__ w2, T ih0, T ih1, T ih2) {
        const int64_t sy = d.g[0], sz = (int64_t)d.g[0] * d.g[1];
        if (KIND == 2) {
            cp[0] = (i + 1 < d.g[0]) ? w0[2 * p] : T(0);
            cm[0] = (i > 0) ? w0[2 * p + 1] : T(0);
            cp[1] = (j + 1 < d.g[1]) ? w1[2 * p] : T(0);
            cm[1] = (j > 0) ? w1[2 * p + 1] : T(0);
            if (DIM == 3) {
                cp[2] = (k + 1 < d.g[2]) ? w2[2 * p] : T(0);
                cm[2] = (k > 0) ? w2[2 * p + 1] : T(0);
            }
        } else if (KIND == 0) {
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
    __device__ __forceinline__ void restrict_support(int I, bool nodal, int nf, bool mixed = false) {
        n = 0;
        if (mixed && !nodal) {
            // eq. tildeRu1: (1/2)[1 * 1], the two fine cells 2I and 2I+1
            idx[0] = 2 * I; wt[0] = 0.5f; idx[1] = 2 * I + 1; wt[1] = 0.5f; n = 2;
            return;
        }
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

// Restriction and prolongation, specialised at compile time on the nodal
// pattern NM of the block (bit a: nodal along axis a) and the dimension.
// 1D restriction along one axis: nodal (1/4)[1 2 1] from fine 2I-1;
// cell-centred full weighting (1/8)[1 3 3 1] from fine 2I-1; cell-centred
// mixed (eq. tildeRu1) (1/2)[1 1] from fine 2I.
template <bool NODAL, bool MIXED = false>
struct R1 {
    static constexpr bool HALF = MIXED && !NODAL;
    static constexpr int S = NODAL ? 3 : (HALF ? 2 : 4);
    static constexpr int FIRST = HALF ? 0 : -1;       // first fine index is 2I + FIRST
    __device__ static constexpr float w(int t) {
        return NODAL ? (t == 1 ? 0.5f : 0.25f) : (HALF ? 0.5f : ((t == 1 || t == 2) ? 0.375f : 0.125f));
    }
};

// Interpolation weights of fine index l along one axis: two coarse indices
// (the second weight may be zero, its index then repeats the first).
template <bool NODAL>
__device__ __forceinline__ void p1(int l, int nc, int& i0, int& i1, float& w0, float& w1) {
    if (NODAL) {
        if ((l & 1) == 0) { i0 = l >> 1; i1 = i0; w0 = 1.0f; w1 = 0.0f; }
        else { i0 = (l - 1) >> 1; i1 = i0 + 1; w0 = 0.5f; w1 = 0.5f; }
    } else {
        i0 = l >> 1; w0 = 0.75f;
        const int nb = (l & 1) ? i0 + 1 : i0 - 1;
        if (nb >= 0 && nb < nc) { i1 = nb; w1 = 0.25f; } else { i1 = i0; w1 = 0.0f; }
    }
}

}  // namespace eh
