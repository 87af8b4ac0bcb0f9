"""Oracle: commutator and the matrices of Theorem 3.1 (dense, tiny grids).

Test infrastructure only (see the package docstring).

* Xi = B A - A_p B (eq. commutator).
* K = D_L H = [A B^T; Xi H_p] (eq. mixed-distributed).
* T = I - P^{-1} K (eq. error_iter_mat) and Z = Xi A^{-1} B^T H_p^{-1}
  (eq. Z).  Theorem 3.1: T has a null space of dimension >= n (n = size of
  A) and spec(T) = spec(Z) united with {0}.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .elastic import ElasticSystem


def commutator(sys: ElasticSystem):
    return (sys.B @ sys.A() - sys.A_p() @ sys.B).tocsr()


def distributed_matrix(sys: ElasticSystem):
    """K = D_L H with D_L = [I 0; B -A_p] (eqs. mixed-distributor,
    mixed-distributed)."""
    nu = sys.nu_total
    DL = sp.bmat([[sp.identity(nu), None], [sys.B, -sys.A_p()]], format="csr")
    return (DL @ sys.H()).tocsr(), DL


def Z_matrix(sys: ElasticSystem):
    """Z = Xi A^{-1} B^T H_p^{-1} (dense)."""
    Xi = commutator(sys).toarray()
    A = sys.A().toarray()
    Bt = sys.B.T.toarray()
    Hp = sys.H_p().toarray()
    return Xi @ np.linalg.solve(A, Bt @ np.linalg.inv(Hp))
