"""Least-squares full-waveform-inversion misfit as a torch.autograd.Function.

Phi(vp, vs, rho) = 1/2 sum_s || P_r u_s - d_s ||^2 with H(vp, vs, rho) u_s = b_s
(the mixed elastic Helmholtz system of the paper, Section 2.1, used as the
forward solver of frequency-domain elastic FWI, Section 4).

forward:  one batched FGMRES solve for all sources (eh_solve), then the
          receiver sampling and the adjoint sources (eh_misfit).
backward: one batched adjoint solve H w_s = conj(P_r^T (P_r u_s - d_s)) --
          H is complex symmetric, so lambda_s = conj(w_s) solves
          H^H lambda_s = P_r^T (P_r u_s - d_s) with the same operator and
          preconditioner -- then the per-cell gradient kernel
          (eh_gradient).  Every arithmetic step runs in libehelm.so; this
          module only moves arguments.
"""
from __future__ import annotations

import math

import torch

from .solver import EhelmError, ElasticHelmholtz


def _require_converged(info, what, tol):
    """A solve that stopped at maxit gives a wrong misfit or gradient:
    refuse it rather than hand it to autograd."""
    bad = [q for q, i in enumerate(info) if not i["converged"]]
    if bad:
        worst = max(info[q]["relres_true"] for q in bad)
        raise EhelmError(1, f"{what} solve did not reach tol {tol:g} for sources {bad} "
                            f"(worst relative residual {worst:.3e})")


class ElasticMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vp, vs, rho, geom, b, rec, d_obs):
        """vp, vs, rho: float64 tensors of the cell shape (x fastest).
        geom: dict with n, h, omega and optional solver settings (levels,
        alpha, mg_precision, restart, abc_width, abc_sides, tol, maxit).
        b: (nsrc, ndof) complex128 CUDA tensor; rec: int64 CUDA tensor of
        receiver dofs; d_obs: (nsrc, nrec) complex128 CUDA tensor."""
        g = dict(geom)
        tol = g.pop("tol", 1e-10)
        maxit = g.pop("maxit", 2000)
        n, h, omega = g.pop("n"), g.pop("h"), g.pop("omega")
        solver = ElasticHelmholtz(n, h, vp.detach().cpu().numpy(), vs.detach().cpu().numpy(),
                                  rho.detach().cpu().numpy(), omega, **g)
        u, info = solver.solve(b, tol=tol, maxit=maxit)
        try:
            _require_converged(info, "forward", tol)
        except EhelmError:
            solver.close()
            raise
        phi, adj_rhs = solver.misfit(u, rec, d_obs)
        ctx.solver = solver
        ctx.tol, ctx.maxit = tol, maxit
        ctx.shape = vp.shape
        ctx.device = vp.device
        ctx.info = info
        ctx.save_for_backward(u, adj_rhs)
        return torch.tensor(phi, dtype=torch.float64, device=vp.device)

    @staticmethod
    def backward(ctx, grad_phi):
        u, adj_rhs = ctx.saved_tensors
        solver = ctx.solver
        w, info = solver.solve(adj_rhs, tol=ctx.tol, maxit=ctx.maxit)
        try:
            _require_converged(info, "adjoint", ctx.tol)
            gvp, gvs, grho = solver.gradient(u, w)
        finally:
            solver.close()
        ctx.adjoint_info = info
        scale = grad_phi.to(gvp.device)
        out = [(scale * t).reshape(ctx.shape).to(ctx.device) for t in (gvp, gvs, grho)]
        return out[0], out[1], out[2], None, None, None, None


def misfit(vp, vs, rho, geom, b, rec, d_obs):
    """Phi(vp, vs, rho); differentiable with respect to vp, vs and rho."""
    return ElasticMisfit.apply(vp, vs, rho, geom, b, rec, d_obs)
