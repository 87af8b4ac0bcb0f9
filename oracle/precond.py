"""Oracle: the block-acoustic preconditioner.

Test infrastructure only (see the package docstring).

Section 3 of the paper.  The left distributor D_L = [I 0; B -A_p]
(eq. mixed-distributor) turns H into K = D_L H = [A B^T; Xi H_p]
(eq. mixed-distributed) and the preconditioner drops the commutator block:
P = [A B^T; 0 H_p] (eq. prec).  One application z = P^{-1} D_L r is

    t   = B r_u - A_p r_p          (corrected right-hand side)
    e_p = H_p^{-1} t               (pressure-velocity acoustic block)
    g   = r_u - B^T e_p
    e_k = A_k^{-1} g_k, k = 1..d    (shear-velocity acoustic blocks)

Each block inverse is either exact (sparse LU, as in Table
scalability_linear) or one multigrid cycle on the shifted block (Section
4.4).  Reading: the shift alpha enters only the blocks that are inverted
(A_k and H_p, all levels); the distributor's A_p and the couplings B, B^T are
unshifted.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .elastic import ElasticSystem, face_nodal
from .multigrid import Hierarchy


class BlockAcoustic:
    def __init__(self, sys: ElasticSystem, alpha=0.0, solver="mg", levels=3,
                 cycle="V", nu=(1, 2), damping=(0.8, 0.8, 0.3),
                 tilde_Ap=False, intergrid="full"):
        self.sys = sys
        d = sys.dim
        self.Ap = sys.A_p_tilde() if tilde_Ap else sys.A_p()
        if tilde_Ap:
            Hp = (sys.BBt() + sys.A_p_tilde(alpha) @ sys.C).tocsr()
        else:
            Hp = sys.H_p(alpha)
        blocks = [sys.A_block(k, alpha) for k in range(d)]
        if solver == "exact":
            lu_p = spla.splu(Hp.tocsc())
            lu_u = [spla.splu(b.tocsc()) for b in blocks]
            self.solve_p = lu_p.solve
            self.solve_u = [lu.solve for lu in lu_u]
        elif solver == "mg":
            cell = tuple(False for _ in range(d))
            self.mg_p = Hierarchy(Hp, sys.n, cell, levels, damping, nu, cycle,
                                  intergrid)
            self.mg_u = [Hierarchy(blocks[k], sys.n, face_nodal(d, k), levels,
                                   damping, nu, cycle, intergrid) for k in range(d)]
            self.solve_p = self.mg_p
            self.solve_u = list(self.mg_u)
        else:
            raise ValueError(solver)
        self.Hp = Hp
        self.blocks = blocks

    def distribute(self, r):
        """Corrected right-hand side t = B r_u - A_p r_p (eq.
        mixed-distributed)."""
        parts = self.sys.split(r)
        ru = np.concatenate(parts[:-1])
        return self.sys.B @ ru - self.Ap @ parts[-1]

    def apply(self, r):
        """z = P^{-1} D_L r."""
        s = self.sys
        parts = s.split(np.asarray(r, dtype=np.complex128))
        t = self.distribute(r)
        ep = self.solve_p(t)
        eu = []
        for k in range(s.dim):
            g = parts[k] - s.Bt[k] @ ep
            eu.append(self.solve_u[k](g))
        return np.concatenate(eu + [ep])

    __call__ = apply
