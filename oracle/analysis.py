"""Oracle: commutator and the matrices of Theorem 3.1 (dense, tiny grids).

Test infrastructure only (see the package docstring).

* Xi = B A - A_p B (eq. commutator).
* K = D_L H = [A B^T; Xi H_p] (eq. mixed-distributed).
* T = I - P^{-1} K (eq. error_iter_mat) and Z = Xi A^{-1} B^T H_p^{-1}
  (eq. Z).  Theorem 3.1: T has a null space of dimension >= n (n = size of
  A) and spec(T) = spec(Z) united with {0}.
* rho(Z) as a function of the shift (Section 5, the power method on a
  mat-vec of Z).  Reading: Z(alpha) = Xi A_alpha^{-1} B^T H_p,alpha^{-1},
  the commutator unshifted and the two inverted blocks shifted as in the
  preconditioner (eq. shift); alpha = 0 is eq. Z.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .elastic import ElasticSystem


def commutator(sys: ElasticSystem):
    return (sys.B @ sys.A() - sys.A_p() @ sys.B).tocsr()


def distributed_matrix(sys: ElasticSystem):
    """K = D_L H with D_L = [I 0; B -A_p] (eqs. mixed-distributor,
    mixed-distributed)."""
    nu = sys.nu_total
    DL = sp.bmat([[sp.identity(nu), None], [sys.B, -sys.A_p()]], format="csr")
    return (DL @ sys.H()).tocsr(), DL


def Z_matrix(sys: ElasticSystem, alpha=0.0):
    """Z(alpha) = Xi A_alpha^{-1} B^T H_p,alpha^{-1} (dense)."""
    Xi = commutator(sys).toarray()
    A = sp.block_diag([sys.A_block(k, alpha) for k in range(sys.dim)]).toarray()
    Bt = sys.B.T.toarray()
    Hp = sys.H_p(alpha).toarray()
    return Xi @ np.linalg.solve(A, Bt @ np.linalg.inv(Hp))


class ZOperator:
    """Matrix-free Z(alpha) v with sparse LU solves for the shifted blocks:
    t = H_p,alpha^{-1} v, g = B^T t, w_k = A_k,alpha^{-1} g_k, Z v = Xi w."""

    def __init__(self, sys: ElasticSystem, alpha=0.0):
        self.sys = sys
        self.Xi = commutator(sys)
        self.lu_p = spla.splu(sys.H_p(alpha).tocsc())
        self.lu_u = [spla.splu(sys.A_block(k, alpha).tocsc()) for k in range(sys.dim)]

    def __call__(self, v):
        s = self.sys
        g = s.B.T @ self.lu_p.solve(np.asarray(v, dtype=np.complex128))
        w, o = [], 0
        for k in range(s.dim):
            n = s.face_sizes[k]
            w.append(self.lu_u[k].solve(g[o:o + n]))
            o += n
        return self.Xi @ np.concatenate(w)


def power_method(op, v0, iters):
    """Power iteration v <- Z v / ||Z v||; returns the sequence of estimates
    ||Z v_k|| of the spectral radius (v_k normalised)."""
    v = np.asarray(v0, dtype=np.complex128)
    v = v / np.linalg.norm(v)
    est = []
    for _ in range(iters):
        y = op(v)
        nrm = np.linalg.norm(y)
        est.append(nrm)
        if nrm == 0.0:
            break
        v = y / nrm
    return np.array(est)
