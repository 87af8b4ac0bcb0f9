"""Oracle: right-preconditioned flexible GMRES(m).

Test infrastructure only (see the package docstring).

The paper runs (flexible) GMRES (Section 2.2, Saad 1993), non-restarted for
Table scalability_linear and restarted as GMRES(5) for the multigrid tables,
stopping at a relative residual below 1e-6 (Section 4).  Readings: the
starting guess is zero, the residual is the unpreconditioned
||b - H x|| / ||b||, and one iteration is one preconditioner application
("preconditioning cycles" in the tables).

Each cycle builds the flexible Arnoldi relation H Z_j = V_{j+1} Hbar_j with
modified Gram-Schmidt and takes y = argmin ||beta e_1 - Hbar_j y|| from a
dense least-squares solve (the plain definition; no Givens rotations), so
the least-squares residual is the residual estimate.  The true residual is
recomputed at every restart and at the end.
"""
from __future__ import annotations

import numpy as np


class Result:
    def __init__(self, x, iters, converged, history, relres_true):
        self.x = x
        self.iters = iters
        self.converged = converged
        self.history = history          # residual estimate after each iteration
        self.relres_true = relres_true


def fgmres(apply_H, apply_M, b, restart=20, tol=1e-6, maxit=1000,
           breakdown_tol=1e-14, record=None):
    """Solve H x = b.  apply_M(v) is the (possibly varying) preconditioner.

    record: optional dict; when given, the Arnoldi quantities (V, Z, Hbar) of
    the last cycle are stored in it for inspection."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return Result(x, 0, True, [], 0.0)
    its = 0
    history = []
    converged = False
    while its < maxit:
        r = b - apply_H(x)
        beta = np.linalg.norm(r)
        if beta / bnorm < tol:
            converged = True
            break
        m = min(restart, maxit - its)
        V = [r / beta]
        Z = []
        Hbar = np.zeros((m + 1, m), dtype=np.complex128)
        j_end = 0
        y = None
        for j in range(m):
            z = apply_M(V[j])
            Z.append(z)
            w = apply_H(z)
            its += 1
            w0 = np.linalg.norm(w)
            for i in range(j + 1):
                Hbar[i, j] = np.vdot(V[i], w)
                w = w - Hbar[i, j] * V[i]
            Hbar[j + 1, j] = np.linalg.norm(w)
            j_end = j + 1
            rhs = np.zeros(j + 2, dtype=np.complex128)
            rhs[0] = beta
            y, *_ = np.linalg.lstsq(Hbar[:j + 2, :j + 1], rhs, rcond=None)
            est = np.linalg.norm(rhs - Hbar[:j + 2, :j + 1] @ y)
            history.append(est / bnorm)
            breakdown = Hbar[j + 1, j].real <= breakdown_tol * max(w0, 1e-300)
            if not breakdown:
                V.append(w / Hbar[j + 1, j])
            if est / bnorm < tol or breakdown or its >= maxit:
                break
        for i in range(j_end):
            x = x + y[i] * Z[i]
        if record is not None:
            record.update(V=V, Z=Z, Hbar=Hbar[:j_end + 1, :j_end], beta=beta)
        if history and history[-1] < tol:
            r = b - apply_H(x)
            if np.linalg.norm(r) / bnorm < tol:
                converged = True
                break
    relres = np.linalg.norm(b - apply_H(x)) / bnorm
    return Result(x, its, converged or relres < tol, history, relres)
