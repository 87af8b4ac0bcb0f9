/*
 * ehelm -- block-acoustic preconditioned solver for the elastic Helmholtz
 * equation in mixed displacement-pressure form on MI355X (gfx950).
 *
 * Method: Yovel & Treister, "A block-acoustic preconditioner for the elastic
 * Helmholtz equation".  The discrete system is the MAC discretisation
 *     H = [A  B^T; B  -C]                           (eq. mixed-discretized)
 * with A = grad_h^T A_e(mu) grad_h - w^2 A_f(rho (1 - i gamma/w)), one
 * acoustic block A_k per displacement component, B = -div_h, B^T = grad_h,
 * C = diag(1/(lambda+mu)).  It is solved by flexible GMRES, right
 * preconditioned by P^{-1} D_L with the distributor D_L = [I 0; B -A_p]
 * (eq. mixed-distributor), A_p = B B^T mu - w^2 M_p (eq. Ap), and the block
 * triangular P = [A B^T; 0 H_p] (eq. prec), H_p = B B^T + A_p C (eq. Hp).
 * Each diagonal block is replaced by one shifted-Laplacian multigrid cycle
 * (eq. shift, Section 4.4.1): damped Jacobi, full-weighting restriction
 * (eqs. Ru1, Rp), (bi/tri)linear prolongation, Galerkin coarse operators
 * (eq. galerkin) and a direct coarsest solve.
 *
 * Conventions shared by every call:
 *  - Grid: n[0] x n[1] (x n[2]) cells, x first; cell sizes h[0..dim-1].
 *  - Vector layout: [u_1 | ... | u_dim | p], each field C-contiguous with x
 *    fastest.  u_k lives on the k-faces: its extent along axis k is n[k]+1.
 *    p lives at cell centres.  ndof = sum of the field sizes (eh_ndof).
 *  - Complex numbers are interleaved (re, im) doubles ("complex128").
 *  - Several right-hand sides are stored one after the other
 *    (RHS-major, leading dimension ndof).
 *  - Buffers passed as `void *` are DEVICE pointers owned by the caller;
 *    `const double *` medium arrays are HOST pointers, copied during create.
 *  - All work is enqueued on the context's HIP stream.  Calls return after
 *    enqueue, except eh_create, eh_solve and eh_gradient which synchronise.
 *    eh_solve runs on a stream of its own, ordered after the context's
 *    stream, and returns when its work is complete.
 *  - Errors are returned as status codes; nothing throws across this
 *    boundary and nothing exits.  eh_last_error gives a message.  Argument
 *    errors are detected before any device work and leave no side effects.
 */
#ifndef EHELM_H
#define EHELM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eh_ctx eh_ctx;

typedef enum {
    EH_OK = 0,
    EH_NOT_CONVERGED = 1,   /* warning: outputs valid, tolerance not reached */
    EH_ERR_ARG = -1,        /* invalid argument; nothing was done            */
    EH_ERR_HIP = -2,        /* HIP runtime error                             */
    EH_ERR_OOM = -3,        /* device allocation failed                      */
    EH_ERR_STATE = -4       /* context unusable (earlier error)              */
} eh_status;

/* Solver options.  eh_default_opts fills the paper's 2D defaults. */
typedef struct {
    int levels;             /* multigrid levels per block (>= 1); each n[a] must be divisible by 2^(levels-1) */
    int cycle;              /* 0 = V-cycle (one recursive call), 1 = W-cycle (two), Algorithm TwoCycle */
    int nu_pre, nu_post;    /* damped-Jacobi sweeps before / after the coarse correction; paper: (1,2) in 2D, (2,2) in 3D */
    int n_damping;          /* number of entries used in damping[] (>= 1); the last is repeated on deeper levels */
    double damping[8];      /* Jacobi damping per level; paper: 0.8, 0.8, 0.3 (2D), 0.8, 0.8, 0.2 (3D) */
    double alpha;           /* shift of eq. shift: extra attenuation gamma/w -> gamma/w + alpha in the inverted blocks */
    int mg_precision;       /* 32: complex64 multigrid, 64: complex128 multigrid; coarsest solve always FP64 */
    int restart;            /* FGMRES restart length m (>= 1) */
    int abc_width;          /* absorbing layer width in cells (Section 4: 20) */
    unsigned abc_sides;     /* bitmask of absorbing sides: bit 2a low side of axis a, bit 2a+1 high side */
    double gamma0;          /* natural attenuation everywhere (Section 4: 0.01 pi) */
    int intergrid;          /* 0: full-weighting restriction R = P^T/2^d (eqs. Ru1, Rp);
                               1: mixed intergrid, (1/2)[1 * 1] along cell-centred axes
                               (eq. tildeRu1, the paper's 3D setting); P is (bi/tri)linear either way */
    int graphs;             /* 1: eh_solve captures each Arnoldi step (preconditioner, operator, first
                               Gram-Schmidt pass) as a HIP graph once and replays it; 0: plain launches.
                               While a kernel class is timed (eh_timer_enable) plain launches are used. */
    int autotune;           /* 1: at the first solve / preconditioner call for a batch size, time every
                               candidate workgroup shape of the sweep, restriction and prolongation kernels
                               (with fused legs: every tile configuration of each level's down and up leg)
                               per level and block group and keep the fastest (results are unchanged);
                               choices are cached in the file named by $EH_TUNE_CACHE when set */
    int fused;              /* 1: 2D V(1,nu_post) cycles (nu_post 1 or 2) from a zero guess run each level
                               as two LDS-tiled launches -- the restricted residual of the first sweep
                               (down leg) and prolongation + correction + all post-sweeps (up leg);
                               0: one launch per sweep and transfer.  Same arithmetic per point;
                               summation order may differ. */
    int ap_variant;         /* 0: A_p = B B^T diag(mu) - w^2 M_p (eq. Ap) in the distributor and in
                               H_p = B B^T + A_p C (eq. Hp), the paper's choice; 1: the alternative of the
                               Remark after eq. prec, A~_p = B A_f(mu) B^T - w^2 M_p, in both */
    int coarse_solver;      /* direct solve of the coarsest level (Section 4.4.1), FP64 either way:
                               1: explicit dense inverse (Gauss-Jordan, partial pivoting), applied as a
                                  matrix-vector product; at most 6000 points per block;
                               2: block-tridiagonal LU over groups of planes (lines in 2D) normal to one
                                  axis, each group as wide as the coarse stencil's half width along it;
                                  Schur complements inverted by blocked Gauss-Jordan (partial pivoting
                                  inside 32 x 32 pivot blocks), applied as a forward and a back sweep of
                                  one launch per group; the factors are checked at create by one solve
                                  whose FP64 residual must stay below 1e-8 (EH_ERR_ARG otherwise);
                               0: 1 while every block's coarsest grid has at most 6000 points, else 2 */
    int drop_converged;     /* 1: at each FGMRES restart, right-hand sides whose true residual is below tol
                               leave the batch -- the others are gathered into the first slots and every
                               later launch covers only them (two ndof-vectors per remaining right-hand side
                               are allocated at the first such restart and freed before eh_solve returns);
                               per right-hand side the arithmetic, the result and the iteration count are
                               the same as with 0, where every launch covers the whole batch */
} eh_opts;

typedef struct {
    int iters;              /* preconditioner applications (the paper's "preconditioning cycles") */
    int converged;          /* 1 if the true relative residual is below tol */
    double relres_true;     /* ||b - H x|| / ||b||, recomputed in FP64 at the end */
    double relres_est;      /* FGMRES least-squares estimate at the last iteration */
} eh_info;

/* Fill `opts` with defaults: 3 levels, V(1,2), damping 0.8/0.8/0.3,
 * alpha 0.1, complex64 multigrid, restart 20, 20-cell layer on all sides but
 * the top, gamma0 = 0.01 pi, full-weighting intergrid, automatic choice of
 * the coarsest solver (Sections 4 and 4.4.1). */
void eh_default_opts(eh_opts *opts);

/* Set up the operator and the preconditioner for one grid, medium and
 * frequency (Section 2.1, eq. mixed-discretized; Section 4 for the absorbing
 * layer).  dim is 2 or 3.  vp, vs, rho: host arrays of n[0]*...*n[dim-1]
 * cell values (x fastest), requiring vp > vs > 0 and rho > 0 (so that
 * mu = rho vs^2 > 0 and lambda + mu = rho (vp^2 - vs^2) > 0).  omega > 0.
 * hip_stream: a hipStream_t (NULL = default stream).  On success *ctx owns
 * all device memory of the hierarchy; free it with eh_destroy. */
eh_status eh_create(eh_ctx **ctx, int dim, const int64_t *n, const double *h,
                    const double *vp, const double *vs, const double *rho,
                    double omega, const eh_opts *opts, void *hip_stream);

/* Number of unknowns per right-hand side. */
int64_t eh_ndof(const eh_ctx *ctx);

/* y = H x for nrhs vectors (eq. mixed-discretized), complex128 device
 * buffers of nrhs*ndof entries; x and y must not overlap. */
eh_status eh_apply_operator(eh_ctx *ctx, const void *x, void *y, int nrhs);

/* z = P^{-1} D_L r: one application of the block-acoustic preconditioner
 * (eqs. mixed-distributed and prec) with one multigrid cycle per block,
 * in the context's multigrid precision; r and z are complex128 device
 * buffers of nrhs*ndof entries and must not overlap. */
eh_status eh_apply_preconditioner(eh_ctx *ctx, const void *r, void *z, int nrhs);

/* One multigrid cycle (Algorithm TwoCycle, recursive) on one shifted block:
 * block 0..dim-1 is A_{block+1} on its faces, block dim is H_p on the cells.
 * e ~ X_s^{-1} f with a zero initial guess.  f and e are complex128 device
 * buffers of nrhs * (points of the block) entries. */
eh_status eh_block_cycle(eh_ctx *ctx, int block, const void *f, void *e, int nrhs);

/* y = X x with the shifted block operator of `block` on multigrid level
 * `level` (level 0 = fine grid; deeper levels are the Galerkin operators of
 * eq. galerkin), evaluated in the multigrid precision.  complex128 device
 * buffers of nrhs * (points of that level) entries. */
eh_status eh_block_apply(eh_ctx *ctx, int block, int level, const void *x, void *y, int nrhs);

/* Points per axis of a block's grid on a level (out[0..2]; 1 for unused axes). */
eh_status eh_block_dims(const eh_ctx *ctx, int block, int level, int64_t *out);

/* Solve H x = b for nrhs right-hand sides with right-preconditioned
 * FGMRES(restart) (Section 2.2, flexible GMRES), starting from x = 0,
 * stopping each right-hand side when ||b - H x||/||b|| < tol or after maxit
 * preconditioner applications.  b, x: complex128 device buffers of
 * nrhs*ndof entries.  info: host array of nrhs entries (may be NULL);
 * relres_true is recomputed in FP64 from the returned x.  The Arnoldi
 * bookkeeping runs on the device; iteration counts may differ by one from
 * an implementation with modified Gram-Schmidt (this one uses classical
 * Gram-Schmidt applied twice).  Returns EH_NOT_CONVERGED if any right-hand
 * side missed tol, EH_ERR_STATE if a non-finite value appeared (x is then
 * unspecified).  Synchronises. */
eh_status eh_solve(eh_ctx *ctx, const void *b, void *x, int nrhs, double tol,
                   int maxit, eh_info *info);

/* Solve one shifted acoustic block alone, X_b x = f on the fine grid
 * (block 0..dim-1: A_{b+1}, block dim: H_p; the operators the
 * preconditioner inverts, eq. shift), with FGMRES(restart) right-
 * preconditioned by the block's multigrid cycle.  The operator is applied
 * in the multigrid precision.  f, x: complex128 device buffers of
 * nrhs * (points of the block) entries; info as for eh_solve.
 * Synchronises.  Returns EH_NOT_CONVERGED if any right-hand side missed
 * tol. */
eh_status eh_block_solve(eh_ctx *ctx, int block, const void *f, void *x, int nrhs,
                         double tol, int maxit, eh_info *info);

/* y = Z(alpha) v for one cell vector: Z = Xi A^-1 B^T H_p^-1 (eq. Z,
 * Theorem 3.1) with the commutator Xi = B A - A_p B (eq. commutator;
 * B A - A~_p B when ap_variant = 1) and the inverses of the shifted
 * blocks the preconditioner uses (alpha = 0 gives eq. Z exactly).  Each
 * inverse is an eh_block_solve to tol (at most maxit iterations).  v, y:
 * complex128 device buffers of n_cells entries.  Synchronises; returns
 * EH_NOT_CONVERGED if an inner solve missed tol. */
eh_status eh_apply_Z(eh_ctx *ctx, const void *v, void *y, double tol, int maxit);

/* Power method for the spectral radius of Z(alpha) (Section 5, rho(Z) as a
 * function of the shift): v <- Z v / ||Z v||, starting from the caller's
 * v (device, n_cells complex128, normalised first, overwritten by the last
 * iterate); est[k] = ||Z v_k|| for k < iters (host array).  Inner solves as
 * eh_apply_Z.  Synchronises. */
eh_status eh_power_Z(eh_ctx *ctx, void *v, int iters, double tol, int maxit, double *est);

/* Gradient of Phi = 1/2 sum_s ||P_r u_s - d_s||^2 with respect to per-cell
 * vp, vs and rho: g_m = -Re sum_s lam_s^H (dH/dm) u_s, with dH/dm from the
 * assembly of eq. mixed-discretized (mu through the cell and edge averages,
 * rho through the face mass, lambda+mu through C; gamma and omega held
 * fixed; chain rule mu = rho vs^2, lambda+mu = rho (vp^2 - vs^2)).
 * H is complex symmetric, so the adjoint fields are lam_s = conj(w_s) where
 * H w_s = conj(P_r^T (P_r u_s - d_s)) -- the right-hand side eh_misfit
 * writes -- and this call takes w directly.
 * u, w: complex128 device buffers of nrhs*ndof entries; g_vp, g_vs, g_rho:
 * device double buffers of n_cells entries (overwritten).  Synchronises. */
eh_status eh_gradient(eh_ctx *ctx, const void *u, const void *w, int nrhs,
                      double *g_vp, double *g_vs, double *g_rho);

/* Receiver sampling for the misfit: given fields u (nrhs*ndof complex128,
 * device), receiver dof indices rec (nrec int64, device, each in
 * [0, ndof)) and observed data d (nrhs*nrec complex128, device, receiver
 * fastest), writes conj(P_r^T (P_r u_s - d_s)) -- the right-hand side of
 * the adjoint solve -- into g (nrhs*ndof complex128, device) and returns
 * Phi in *phi (host).  Synchronises. */
eh_status eh_misfit(eh_ctx *ctx, const void *u, const int64_t *rec, int nrec,
                    const void *d, int nrhs, void *g, double *phi);

/* eh_misfit for callers that cannot allocate device memory or wait: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same misfit, adjoint right-hand side g and summation order as
 * eh_misfit (bitwise the same results), with three differences: phi is a
 * DEVICE pointer to one double, written on the context's stream; the call
 * only enqueues (no allocation, no synchronisation, no hipMemset: g is
 * cleared by a kernel); receiver indices are checked on the device, and an
 * index outside [0, ndof) is skipped and makes *phi NaN.  The per-source
 * partial sums live in a fixed device array of the library, one per GPU,
 * 4096 doubles (32 KiB) held until the process ends: nrhs above 4096 is
 * EH_ERR_ARG.  Every call on one GPU shares that array and overwrites the
 * entries it uses before reading them; calls that overlap on one GPU (other
 * streams or contexts) race on it. */
eh_status eh_misfit_noalloc(eh_ctx *ctx, const void *u, const int64_t *rec, int nrec,
                            const void *d, int nrhs, void *g, double *phi);

/* Event timing of kernel classes, for measuring achieved bandwidth.
 * Bit c of class_mask selects class c: 0 fine-level Jacobi sweep,
 * 1 fine-level residual, 2 coarse-level (Galerkin stencil) sweeps and
 * residuals, 3 restriction, 4 prolongation, 5 coarsest dense solve,
 * 6 operator apply, 7 distributor, 8 coupling, 9 Krylov vector kernels,
 * 10 fine-level first sweep from a zero guess, 11 fine-level fused down
 * leg, 12 fine-level fused up leg, 13 coarse-level fused down legs, 14
 * coarse-level fused up legs.  While selected, every
 * launch of the class is bracketed by two hipEvents on the context's
 * stream.  0 disables timing. */
eh_status eh_timer_enable(eh_ctx *ctx, unsigned class_mask);

/* Sum, over the launches of class `cls` recorded since the last read, of
 * the event-measured milliseconds and of the algorithmic bytes (each operand
 * read once and each result written once per launch; coefficients counted
 * once per launch, vectors once per right-hand side).  Synchronises on the
 * recorded events and clears them. */
eh_status eh_timer_read(eh_ctx *ctx, int cls, int64_t *launches, double *ms,
                        double *bytes);

/* Replace the stream all later work is enqueued on. */
eh_status eh_set_stream(eh_ctx *ctx, void *hip_stream);

/* Release everything the context owns.  NULL is ignored. */
void eh_destroy(eh_ctx *ctx);

/* Message of the last error on this context (or of the last failed
 * eh_create when ctx is NULL).  Never NULL. */
const char *eh_last_error(const eh_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* EHELM_H */
