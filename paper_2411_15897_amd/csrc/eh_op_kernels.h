// Elastic operator, distributor and coupling kernels (FP64 inputs).
//
//  k_op_face / k_op_cell: y = H x (eq. mixed-discretized).  Rows of u_k:
//      A_k u_k + B_k^T p with B_k^T p = (p(c) - p(c - e_k)) / h_k at the
//      k-face between cells c - e_k and c (zero ghost p outside).
//      Rows of p: B u - C p = -sum_k (u_k(hi face) - u_k(lo face)) / h_k
//      - p / (lambda + mu).
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

// Face (i,j,k) of the k-face grid touches cells with index i_a - 1 and i_a
// along a = kaxis.  Returns the linear cell index of the cell at offset
// `off` (0 or -1) along kaxis, or -1 when it lies outside.
__device__ __forceinline__ int64_t face_cell(const Dims& dc, int kaxis, int i, int j, int k, int off) {
    int c[3] = {i, j, k};
    c[kaxis] += off;
    if (c[kaxis] < 0 || c[kaxis] >= dc.g[kaxis]) return -1;
    return ((int64_t)c[2] * dc.g[1] + c[1]) * dc.g[0] + c[0];
}

// Launch: blockDim (64, 4), gridDim (x tiles, y tiles, planes x chunks of
// the batch); workgroup z takes plane z % planes and right-hand sides
// [c * rch, min(nrhs, c * rch + rch)) with c = z / planes, so a batch on a
// small grid is spread over more workgroups (the arithmetic of each
// right-hand side is unchanged).
//
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

template <class Tin, int DIM, bool RES>
__global__ void __launch_bounds__(256)
k_op_face(Dims d, Dims dc, int kaxis, const double* __restrict__ w0, const double* __restrict__ w1,
          const double* __restrict__ w2, const c128* __restrict__ D0, const cplx<Tin>* __restrict__ u,
          const cplx<Tin>* __restrict__ pf, double ihk, c128* __restrict__ y, int nrhs,
          int64_t vs_in, int64_t vs_out, ResArgs ra, int rch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z % d.g[2];
    const int rlo = (blockIdx.z / d.g[2]) * rch, rhi = min(nrhs, rlo + rch);
    const bool in = i < d.g[0] && j < d.g[1];
    if (!RES && !in) return;
    const int64_t sy = d.g[0], sz = (int64_t)d.g[0] * d.g[1];
    const int64_t p = k * sz + j * sy + i;
    FineCoef<double, 0, DIM> c;
    c128 Dp = mk(0.0, 0.0);
    int64_t chi = -1, clo = -1;
    if (in) {
        c.load(d, i, j, k, p, w0, w1, w2, 0.0, 0.0, 0.0);
        Dp = D0[p];
        chi = face_cell(dc, kaxis, i, j, k, 0);
        clo = face_cell(dc, kaxis, i, j, k, -1);
    }
    for (int r = rlo; r < rhi; ++r) {
        c128 yv = mk(0.0, 0.0);
        if (in) {
            const cplx<Tin>* ur = u + r * vs_in;
            const cplx<Tin>* pr = pf + r * vs_in;
            // off-diagonal sum in FP64
            c128 s = mk(0.0, 0.0);
            if (i + 1 < d.g[0]) s = s + c.cp[0] * ccast<double>(ur[p + 1]);
            if (i > 0) s = s + c.cm[0] * ccast<double>(ur[p - 1]);
            if (j + 1 < d.g[1]) s = s + c.cp[1] * ccast<double>(ur[p + sy]);
            if (j > 0) s = s + c.cm[1] * ccast<double>(ur[p - sy]);
            if (DIM == 3) {
                if (k + 1 < d.g[2]) s = s + c.cp[2] * ccast<double>(ur[p + sz]);
                if (k > 0) s = s + c.cm[2] * ccast<double>(ur[p - sz]);
            }
            c128 g = mk(0.0, 0.0);
            if (chi >= 0) g = g + ccast<double>(pr[chi]);
            if (clo >= 0) g = g - ccast<double>(pr[clo]);
            yv = Dp * ccast<double>(ur[p]) - s + ihk * g;
            if (RES) yv = ra.b[r * vs_out + p] - yv;
            y[r * vs_out + p] = yv;
        }
        if (RES) res_partial(ra, r, k, yv.re * yv.re + yv.im * yv.im);
    }
}

template <class Tin, int DIM, bool RES>
__global__ void __launch_bounds__(256)
k_op_cell(Dims dc, const cplx<Tin>* __restrict__ u0, const cplx<Tin>* __restrict__ u1,
          const cplx<Tin>* __restrict__ u2, const cplx<Tin>* __restrict__ pf,
          const double* __restrict__ C, double ih0, double ih1, double ih2, c128* __restrict__ y,
          int nrhs, int64_t vs_in, int64_t vs_out, ResArgs ra, int rch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z % dc.g[2];
    const int rlo = (blockIdx.z / dc.g[2]) * rch, rhi = min(nrhs, rlo + rch);
    const bool in = i < dc.g[0] && j < dc.g[1];
    if (!RES && !in) return;
    const int64_t p = ((int64_t)k * dc.g[1] + j) * dc.g[0] + i;
    // face-grid strides: u0 grid (g0+1, g1, g2), u1 (g0, g1+1, g2), u2 (g0, g1, g2+1)
    const int64_t f0 = ((int64_t)k * dc.g[1] + j) * (dc.g[0] + 1) + i;
    const int64_t f1 = ((int64_t)k * (dc.g[1] + 1) + j) * dc.g[0] + i;
    const int64_t f2 = ((int64_t)k * dc.g[1] + j) * dc.g[0] + i;
    const int64_t s2 = (int64_t)dc.g[0] * dc.g[1];
    const double Cp = in ? C[p] : 0.0;
    for (int r = rlo; r < rhi; ++r) {
        c128 yv = mk(0.0, 0.0);
        if (in) {
            const int64_t o = r * vs_in;
            c128 div = ih0 * (ccast<double>(u0[o + f0 + 1]) - ccast<double>(u0[o + f0]));
            div = div + ih1 * (ccast<double>(u1[o + f1 + dc.g[0]]) - ccast<double>(u1[o + f1]));
            if (DIM == 3) div = div + ih2 * (ccast<double>(u2[o + f2 + s2]) - ccast<double>(u2[o + f2]));
            const c128 pv = ccast<double>(pf[o + p]);
            yv = mk(-div.re - Cp * pv.re, -div.im - Cp * pv.im);
            if (RES) yv = ra.b[r * vs_out + p] - yv;
            y[r * vs_out + p] = yv;
        }
        if (RES) res_partial(ra, r, k, yv.re * yv.re + yv.im * yv.im);
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
