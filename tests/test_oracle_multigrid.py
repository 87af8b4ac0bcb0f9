"""Pins of the oracle's multigrid (CPU only): the paper's restriction
stencils (eqs. Ru1, Rp), exactness of linear interpolation, the Galerkin
two-grid projection identity and textbook V-cycle contraction."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle.elastic import ElasticSystem, face_nodal
from oracle.multigrid import Hierarchy, prolong_1d, transfer

GOLD = os.path.join(os.path.dirname(__file__), "golden", "intergrid_stencils.json")


def test_restriction_stencils_match_paper():
    g = json.load(open(GOLD))
    # 2D u1 block: nodal in x, cell-centred in y (eq. Ru1)
    n = (8, 8)
    _, R = transfer(n, (True, False))
    nxc, nyc = n[0] // 2 + 1, n[1] // 2
    I, J = 2, 2                                  # interior coarse point
    row = R.getrow(J * nxc + I).toarray().reshape(n[1], n[0] + 1)
    expect = np.zeros_like(row)
    for a, wy in enumerate(g["cell_centred"]):
        for b, wx in enumerate(g["nodal"]):
            expect[2 * J - 1 + a, 2 * I - 1 + b] = wy * wx
    np.testing.assert_allclose(row, expect, atol=1e-15)
    assert row.astype(bool).sum() == g["nnz_R_u"]
    # p block (eq. Rp)
    _, Rp = transfer(n, (False, False))
    row = Rp.getrow(J * (n[0] // 2) + I).toarray().reshape(n[1], n[0])
    expect = np.zeros_like(row)
    for a, wy in enumerate(g["cell_centred"]):
        for b, wx in enumerate(g["cell_centred"]):
            expect[2 * J - 1 + a, 2 * I - 1 + b] = wy * wx
    np.testing.assert_allclose(row, expect, atol=1e-15)
    assert row.astype(bool).sum() == g["nnz_R_p"]


@pytest.mark.parametrize("nodal", [True, False])
def test_prolongation_reproduces_linear_fields(nodal):
    nc = 8
    P = prolong_1d(nc, nodal).toarray()
    if nodal:
        xc, xf = np.arange(nc + 1) * 2.0, np.arange(2 * nc + 1) * 1.0
        inner = slice(None)
    else:
        xc, xf = (np.arange(nc) + 0.5) * 2.0, np.arange(2 * nc) + 0.5
        inner = slice(1, -1)      # the two end cells see a zero ghost
    for f in (np.ones_like, lambda x: 3.0 * x - 1.0):
        np.testing.assert_allclose((P @ f(xc))[inner], f(xf)[inner], atol=1e-13)


def _block(n, alpha, seed=0, omega=0.8):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    vp = rng.uniform(2.0, 3.0, shape)
    vs = vp * 0.5
    rho = rng.uniform(1.0, 2.0, shape)
    return ElasticSystem(n, (1.0,) * len(n), vp, vs, rho, omega=omega,
                         abc_width=2, abc_sides=W.ABC_ALL[len(n)])


@pytest.mark.parametrize("which", ["u1", "p"])
def test_two_grid_projection_identity(which):
    """With Galerkin coarsening the coarse-grid correction is a projection:
    (I - P X_c^{-1} R X) P = 0."""
    n = (12, 8)
    s = _block(n, 0.3)
    if which == "u1":
        X, nodal = s.A_block(0, 0.3), face_nodal(2, 0)
    else:
        X, nodal = s.H_p(0.3), (False, False)
    P, R = transfer(n, nodal)
    Xc = (R @ X @ P).toarray()
    Pd, Rd, Xd = P.toarray(), R.toarray(), X.toarray()
    E = Pd - Pd @ np.linalg.solve(Xc, Rd @ Xd @ Pd)
    assert np.abs(E).max() <= 1e-11 * np.abs(Pd).max()


@pytest.mark.parametrize("which", ["u1", "u2", "p"])
def test_vcycle_contraction_poisson_like(which):
    """Damped-Jacobi V(1,2) on a near-Poisson block (tiny frequency, large
    shift) contracts the error by well under 0.3 per cycle -- textbook
    multigrid behaviour that a wrong transfer or coarse operator destroys."""
    n = (32, 32)
    s = _block(n, 1.0, omega=0.05)
    if which == "p":
        X, nodal = s.H_p(1.0), (False, False)
    else:
        k = 0 if which == "u1" else 1
        X, nodal = s.A_block(k, 1.0), face_nodal(2, k)
    mg = Hierarchy(X, n, nodal, levels=4, damping=(0.8, 0.8, 0.8))
    rng = np.random.default_rng(3)
    x_true = rng.standard_normal(X.shape[0]) + 1j * rng.standard_normal(X.shape[0])
    f = X @ x_true
    x = np.zeros_like(f)
    errs = []
    for _ in range(8):
        x = x + mg(f - X @ x)
        errs.append(np.linalg.norm(x - x_true))
    rate = (errs[-1] / errs[2]) ** (1.0 / 5)
    assert rate < 0.3, rate


def test_coarsest_level_is_exact():
    """A single-level hierarchy is the direct solve."""
    n = (8, 6)
    s = _block(n, 0.2)
    X = s.H_p(0.2)
    mg = Hierarchy(X, n, (False, False), levels=1)
    f = np.arange(X.shape[0]) + 1j
    np.testing.assert_allclose(X @ mg(f), f, rtol=1e-12)


def test_galerkin_operator_is_symmetric_for_Ak():
    """R = P^T / 2^d keeps the complex symmetry of A_k on every level."""
    n = (16, 16)
    s = _block(n, 0.3)
    mg = Hierarchy(s.A_block(1, 0.3), n, face_nodal(2, 1), levels=3)
    for op in mg.ops:
        assert abs(op - op.T).max() <= 1e-12 * abs(op).max()


def test_mixed_restriction_stencils_match_paper():
    """eq. tildeRu1: R~_u1 = 1/4[1 2 1] (x) 1/2[1 * 1] (6 nonzeros per row),
    R~_p = 1/2[1 * 1] (x) 1/2[1 * 1] (4 nonzeros)."""
    g = json.load(open(GOLD))
    n = (8, 8)
    _, R = transfer(n, (True, False), "mixed")
    nxc = n[0] // 2 + 1
    I, J = 2, 2
    row = R.getrow(J * nxc + I).toarray().reshape(n[1], n[0] + 1)
    expect = np.zeros_like(row)
    for a, wy in enumerate(g["mixed_cell_centred"]):
        for b, wx in enumerate(g["nodal"]):
            expect[2 * J + a, 2 * I - 1 + b] = wy * wx
    np.testing.assert_allclose(row, expect, atol=1e-15)
    assert row.astype(bool).sum() == g["nnz_Rt_u"]
    _, Rp = transfer(n, (False, False), "mixed")
    row = Rp.getrow(J * (n[0] // 2) + I).toarray().reshape(n[1], n[0])
    assert row.astype(bool).sum() == g["nnz_Rt_p"]
    np.testing.assert_allclose(row[2 * J:2 * J + 2, 2 * I:2 * I + 2], 0.25)


@pytest.mark.parametrize("which", ["u1", "p"])
def test_mixed_galerkin_projection_and_27_point_stencil(which):
    """With R~ the coarse-grid correction is still a projection
    ((I - P X_c^-1 R~ X) P = 0), and the 3D Galerkin operators stay 27-point
    (3 wide per axis) on every level."""
    n = (8, 8, 8)
    s = _block(n, 0.3)
    if which == "u1":
        X, nodal = s.A_block(0, 0.3), face_nodal(3, 0)
    else:
        X, nodal = s.H_p(0.3), (False, False, False)
    P, R = transfer(n, nodal, "mixed")
    Xc = (R @ X @ P).toarray()
    Pd, Rd, Xd = P.toarray(), R.toarray(), X.toarray()
    E = Pd - Pd @ np.linalg.solve(Xc, Rd @ Xd @ Pd)
    assert np.abs(E).max() <= 1e-11 * np.abs(Pd).max()
    mg = Hierarchy(X, n, nodal, 3, intergrid="mixed")
    for op in mg.ops[1:]:
        assert np.diff(op.tocsr().indptr).max() <= 27
