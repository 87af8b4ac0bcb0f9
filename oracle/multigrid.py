"""Oracle: shifted-Laplacian geometric multigrid for one acoustic block.

Test infrastructure only (see the package docstring).

Follows Section 4.4.1 of the paper ("Multigrid setup") and Algorithm
TwoCycle:

* restriction per block is a Kronecker product of 1D full-weighting
  stencils, (1/4)[1 2 1] along a nodal axis and (1/8)[1 3 * 3 1] along a
  cell-centred axis (eqs. Ru1, Rp);
* prolongation is (bi/tri)linear interpolation.  The paper writes
  P = 2 R^T per 1D factor; in d dimensions that is P = 2^d R^T, i.e.
  R = P^T / 2^d.  Galerkin coarsening makes the cycle invariant to the scale
  of P, so this reading changes nothing but the size of the coarse
  operators;
* coarse operators X_H = R X_h P (eq. galerkin);
* damped Jacobi with damping 0.8, 0.8, 0.3 on levels 1, 2, 3 (last value
  repeated deeper; the coarsest level is solved, never smoothed);
* the coarsest problem is solved directly by LU;
* a V-cycle makes one recursive call, a W-cycle two.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .elastic import kron_axes


def prolong_1d(nc, nodal):
    """1D interpolation from a coarse grid of nc cells to the fine grid of
    2 nc cells.

    nodal: coarse node I sits on fine node 2I; fine node 2I+1 is the mean of
    coarse nodes I and I+1.  Shape (2nc+1) x (nc+1).
    cell-centred: fine cell 2I takes 3/4 of coarse cell I and 1/4 of coarse
    cell I-1, fine cell 2I+1 takes 3/4 of I and 1/4 of I+1; coarse cells
    outside the domain are dropped (zero ghost).  Shape 2nc x nc."""
    rows, cols, vals = [], [], []
    if nodal:
        for I in range(nc + 1):
            rows.append(2 * I); cols.append(I); vals.append(1.0)
        for I in range(nc):
            rows += [2 * I + 1, 2 * I + 1]
            cols += [I, I + 1]
            vals += [0.5, 0.5]
        shape = (2 * nc + 1, nc + 1)
    else:
        for I in range(nc):
            for f, nb in ((2 * I, I - 1), (2 * I + 1, I + 1)):
                rows.append(f); cols.append(I); vals.append(0.75)
                if 0 <= nb < nc:
                    rows.append(f); cols.append(nb); vals.append(0.25)
        shape = (2 * nc, nc)
    return sp.csr_matrix((vals, (rows, cols)), shape=shape)


def restrict_mixed_1d(nc, nodal):
    """1D restriction of the mixed intergrid (eq. tildeRu1): along a nodal
    axis (1/4)[1 2 1] as in full weighting, along a cell-centred axis
    (1/2)[1 * 1], the mean of the two fine cells 2I and 2I+1."""
    rows, cols, vals = [], [], []
    if nodal:
        for I in range(nc + 1):
            for f, w in ((2 * I - 1, 0.25), (2 * I, 0.5), (2 * I + 1, 0.25)):
                if 0 <= f <= 2 * nc:
                    rows.append(I); cols.append(f); vals.append(w)
        shape = (nc + 1, 2 * nc + 1)
    else:
        for I in range(nc):
            rows += [I, I]; cols += [2 * I, 2 * I + 1]; vals += [0.5, 0.5]
        shape = (nc, 2 * nc)
    return sp.csr_matrix((vals, (rows, cols)), shape=shape)


def transfer(n_fine, nodal, intergrid="full"):
    """(P, R) between the grid with n_fine cells per axis and the grid with
    half as many; `nodal[a]` says whether the block's unknowns are nodal
    along axis a.  P is (bi/tri)linear interpolation.  intergrid "full":
    R = P^T / 2^d (eqs. Ru1, Rp); "mixed": R is the Kronecker product of the
    1D restrictions of eq. tildeRu1 (the paper's 3D setting, Section 4.5)."""
    d = len(n_fine)
    for v in n_fine:
        if v % 2:
            raise ValueError("grid not divisible by 2")
    P = kron_axes([prolong_1d(n_fine[a] // 2, nodal[a]) for a in range(d)])
    if intergrid == "full":
        R = (P.T / (2.0 ** d)).tocsr()
    elif intergrid == "mixed":
        R = kron_axes([restrict_mixed_1d(n_fine[a] // 2, nodal[a]) for a in range(d)])
    else:
        raise ValueError(intergrid)
    return P, R


class Hierarchy:
    """Galerkin hierarchy of one block X on `levels` grids."""

    def __init__(self, X, n, nodal, levels, damping=(0.8, 0.8, 0.3),
                 nu=(1, 2), cycle="V", intergrid="full"):
        if levels < 1:
            raise ValueError("levels >= 1")
        self.ops = [sp.csr_matrix(X)]
        self.P, self.R = [], []
        nl = tuple(n)
        for _ in range(levels - 1):
            P, R = transfer(nl, nodal, intergrid)
            self.P.append(P)
            self.R.append(R)
            self.ops.append((R @ self.ops[-1] @ P).tocsr())
            nl = tuple(v // 2 for v in nl)
        self.diag = [op.diagonal() for op in self.ops]
        self.lu = spla.splu(self.ops[-1].tocsc())
        self.damping = tuple(damping)
        self.nu = tuple(nu)
        self.cycle_type = cycle
        self.levels = levels

    def damp(self, level):
        return self.damping[min(level, len(self.damping) - 1)]

    def relax(self, level, f, u):
        """One damped Jacobi sweep u <- u + w_l D^-1 (f - X u)."""
        X, D = self.ops[level], self.diag[level]
        return u + self.damp(level) * (f - X @ u) / D

    def cycle(self, f, level=0, u=None):
        """One multigrid cycle for X_level e = f (Algorithm TwoCycle applied
        recursively); u is the initial guess (zero if None)."""
        if level == self.levels - 1:
            return self.lu.solve(f)
        X, D, w = self.ops[level], self.diag[level], self.damp(level)
        nu1, nu2 = self.nu
        if u is None and nu1 > 0:
            u = w * f / D                     # first sweep from a zero guess
            pre = nu1 - 1
        else:
            if u is None:
                u = np.zeros_like(f)
            pre = nu1
        for _ in range(pre):
            u = self.relax(level, f, u)
        rc = self.R[level] @ (f - X @ u)
        ncalls = 1 if self.cycle_type == "V" else 2
        ec = None
        for _ in range(ncalls):
            ec = self.cycle(rc, level + 1, ec)
        u = u + self.P[level] @ ec
        for _ in range(nu2):
            u = self.relax(level, f, u)
        return u

    def __call__(self, f):
        return self.cycle(f)
