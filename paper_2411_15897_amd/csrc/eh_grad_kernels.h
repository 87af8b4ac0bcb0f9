// Full-waveform-inversion gradient and misfit kernels (FP64).
//
// For the least-squares misfit Phi = 1/2 sum_s ||P_r u_s - d_s||^2 with
// H u_s = b_s, dPhi/dm = -Re sum_s lam_s^H (dH/dm) u_s where
// H^H lam_s = P_r^T (P_r u_s - d_s).  H is complex symmetric, so the adjoint
// fields are lam_s = conj(w_s) with H w_s = conj(P_r^T (P_r u_s - d_s)): the
// same operator and preconditioner serve the adjoint solve.  With
// conj(lam_s) = w_s the per-cell terms are, from the assembly of H
// (eq. mixed-discretized):
//   mu:        sum_k (D_k w_k)(D_k u_k) at the cell, plus for every edge
//              (node in 2D) touching the cell the edge term
//              (G w_k)(G u_k) / (number of cells averaged at that edge);
//   rho:       -w^2 (1 - i gamma/w) sum over the faces f touching the cell
//              of w_f u_f / (number of cells averaged at f);
//   lambda+mu: w_p u_p / (lambda+mu)^2   (from -C = -diag(1/(lambda+mu))).
// The chain rule mu = rho vs^2, lambda + mu = rho (vp^2 - vs^2) gives the
// gradients with respect to vp, vs and rho.
#pragma once

#include "eh_common.h"

namespace eh {

struct GradGeom {
    int n[3];
    double ih[3];
    int64_t off[4];     // field offsets in a vector
    int dim;
};

// value of field k (face grid, nodal along k) at face index f (x-first), or 0
// outside the grid
__device__ __forceinline__ c128 face_val(const GradGeom& G, const c128* v, int k, int f0, int f1, int f2) {
    const int f[3] = {f0, f1, f2};
    int g[3] = {G.n[0], G.n[1], G.n[2]};
    g[k] += 1;
    for (int a = 0; a < 3; ++a)
        if (f[a] < 0 || f[a] >= g[a]) return mk(0.0, 0.0);
    return v[G.off[k] + ((int64_t)f[2] * g[1] + f[1]) * g[0] + f[0]];
}

template <int DIM>
__global__ void __launch_bounds__(256)
k_gradient(GradGeom G, const c128* __restrict__ u, const c128* __restrict__ w, int nrhs, int64_t vs,
           double omega, const double* __restrict__ gamma, const double* __restrict__ lm,
           const double* __restrict__ vp, const double* __restrict__ vsv, const double* __restrict__ rho,
           double* __restrict__ gvp, double* __restrict__ gvs, double* __restrict__ grho) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int l = blockIdx.z;
    if (i >= G.n[0] || j >= G.n[1]) return;
    const int c[3] = {i, j, l};
    const int64_t p = ((int64_t)l * G.n[1] + j) * G.n[0] + i;
    double Tmu = 0.0, Tlm = 0.0, Trho_re = 0.0, Trho_im = 0.0;
    for (int s = 0; s < nrhs; ++s) {
        const c128* U = u + s * vs;
        const c128* Wv = w + s * vs;
        for (int k = 0; k < DIM; ++k) {
            // cell term: derivative of u_k along k at this cell
            int fh[3] = {c[0], c[1], c[2]};
            fh[k] += 1;
            const c128 du = G.ih[k] * (face_val(G, U, k, fh[0], fh[1], fh[2]) - face_val(G, U, k, c[0], c[1], c[2]));
            const c128 dw = G.ih[k] * (face_val(G, Wv, k, fh[0], fh[1], fh[2]) - face_val(G, Wv, k, c[0], c[1], c[2]));
            Tmu += (dw * du).re;
            // edge terms: derivative of u_k along a != k, at edges nodal in k and a
            for (int a = 0; a < DIM; ++a) {
                if (a == k) continue;
                for (int ek = c[k]; ek <= c[k] + 1; ++ek)
                    for (int ea = c[a]; ea <= c[a] + 1; ++ea) {
                        // u_k values at cell-centred a-indices ea-1 and ea
                        int q1[3] = {c[0], c[1], c[2]};
                        q1[k] = ek; q1[a] = ea;
                        int q0[3] = {q1[0], q1[1], q1[2]};
                        q0[a] = ea - 1;
                        const c128 gu = G.ih[a] * (face_val(G, U, k, q1[0], q1[1], q1[2]) - face_val(G, U, k, q0[0], q0[1], q0[2]));
                        const c128 gw = G.ih[a] * (face_val(G, Wv, k, q1[0], q1[1], q1[2]) - face_val(G, Wv, k, q0[0], q0[1], q0[2]));
                        const int ck = (ek >= 1) + (ek <= G.n[k] - 1);
                        const int ca = (ea >= 1) + (ea <= G.n[a] - 1);
                        Tmu += (gw * gu).re / double(ck * ca);
                    }
            }
            // faces of u_k touching the cell
            for (int f = c[k]; f <= c[k] + 1; ++f) {
                int q[3] = {c[0], c[1], c[2]};
                q[k] = f;
                const int cnt = (f >= 1) + (f <= G.n[k] - 1);
                const c128 t = face_val(G, Wv, k, q[0], q[1], q[2]) * face_val(G, U, k, q[0], q[1], q[2]);
                Trho_re += t.re / cnt;
                Trho_im += t.im / cnt;
            }
        }
        const c128 tp = Wv[G.off[DIM] + p] * U[G.off[DIM] + p];
        Tlm += tp.re;
    }
    const double l2 = lm[p] * lm[p];
    // Re( -w^2 (1 - i gamma/w) Trho )
    const double om2 = omega * omega;
    const double Trho_full_re = -om2 * (Trho_re + (gamma[p] / omega) * Trho_im);
    const double Gmu = -Tmu;
    const double Glm = -Tlm / l2;
    const double Grho = -Trho_full_re;
    const double a = vp[p], b = vsv[p], r = rho[p];
    gvp[p] = Glm * 2.0 * r * a;
    gvs[p] = Gmu * 2.0 * r * b - Glm * 2.0 * r * b;
    grho[p] = Gmu * b * b + Glm * (a * a - b * b) + Grho;
}

// One block per right-hand side; thread 0 walks the receivers in order
// (duplicates accumulate deterministically).  g (zeroed by the caller)
// receives conj(P_r^T (P_r u - d)); phi_part[s] = 1/2 ||P_r u_s - d_s||^2.
// A receiver index outside [0, ndof) is skipped and makes phi_part[s] NaN.
__global__ void k_misfit(const c128* __restrict__ u, int64_t vs, int64_t ndof, const int64_t* __restrict__ rec,
                         int nrec, const c128* __restrict__ d, c128* __restrict__ g, double* __restrict__ phi_part) {
    const int s = blockIdx.x;
    if (threadIdx.x != 0) return;
    double acc = 0.0;
    bool bad = false;
    for (int t = 0; t < nrec; ++t) {
        const int64_t q = rec[t];
        if (q < 0 || q >= ndof) { bad = true; continue; }
        const c128 res = u[s * vs + q] - d[(int64_t)s * nrec + t];
        acc += cabs2(res);
        g[s * vs + q] = g[s * vs + q] + cconj(res);
    }
    phi_part[s] = bad ? __builtin_nan("") : 0.5 * acc;
}

// phi = sum of the per-source parts in source order (one thread: the same
// order as a sequential host sum).
__global__ void k_misfit_sum(const double* __restrict__ phi_part, int nrhs, double* __restrict__ phi) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int r = 0; r < nrhs; ++r) s += phi_part[r];
    *phi = s;
}

}  // namespace eh
