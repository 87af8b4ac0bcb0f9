"""Pins of the oracle's block-acoustic preconditioner and FGMRES (CPU only):
Theorem 3.1 on small heterogeneous grids, the exact one-iteration solve for
constant media, the block form of eq. precond_system and the iteration
counts the paper prints (Tables scalability_linear and 2Dlinear)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle.analysis import Z_matrix, commutator, distributed_matrix
from oracle.elastic import ElasticSystem
from oracle.fgmres import fgmres
from oracle.precond import BlockAcoustic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def hetero(n, seed=0, omega=1.2, abc=2):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    vp = rng.uniform(2.0, 3.5, shape)
    vs = vp * rng.uniform(0.35, 0.55, shape)
    rho = rng.uniform(1.0, 2.0, shape)
    return ElasticSystem(n, (1.0,) * len(n), vp, vs, rho, omega=omega,
                         abc_width=abc, abc_sides=W.ABC_ALL[len(n)])


def precond_matrix(M, ndof):
    """Columns of the preconditioner map r -> z, applied to the identity."""
    cols = [M.apply(np.eye(ndof, 1, -j).ravel().astype(np.complex128))
            for j in range(ndof)]
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("n", [(12, 10), (4, 4, 3)])
def test_theorem_3_1(n):
    """T = I - (P^{-1} D_L) H has a null space of dimension n_u (the size of
    A) and spec(T) minus {0} equals spec(Z) minus {0}, Z = Xi A^-1 B^T H_p^-1
    (Theorem 3.1).  The preconditioner is the oracle's own application
    routine with exact block solves, read off column by column."""
    s = hetero(n, 1)
    M = BlockAcoustic(s, alpha=0.0, solver="exact")
    Mmat = precond_matrix(M, s.ndof)
    T = np.eye(s.ndof) - Mmat @ s.H().toarray()
    sv = np.linalg.svd(T, compute_uv=False)
    nullity = int(np.sum(sv < 1e-9 * sv[0]))
    assert nullity == s.nu_total
    eT = np.linalg.eigvals(T)
    eZ = np.linalg.eigvals(Z_matrix(s))
    big = lambda e: np.sort_complex(e[np.abs(e) > 1e-8])
    eT, eZ = big(eT), big(eZ)
    assert eT.shape == eZ.shape
    # match each eigenvalue of T to its nearest of Z
    d = np.abs(eT[:, None] - eZ[None, :]).min(axis=1)
    assert d.max() <= 1e-8 * max(1.0, np.abs(eZ).max())
    # rho(T) = rho(Z)
    assert abs(np.abs(eT).max() - np.abs(eZ).max()) <= 1e-9


def test_block_form_of_preconditioned_distributed_system():
    """P^{-1} K = [I - A^-1 B^T H_p^-1 Xi, 0; H_p^-1 Xi, I]
    (eq. precond_system), with P^{-1} D_L read off the oracle routine."""
    n = (8, 6)
    s = hetero(n, 2)
    M = BlockAcoustic(s, alpha=0.0, solver="exact")
    Mmat = precond_matrix(M, s.ndof)
    K, DL = distributed_matrix(s)
    # M = P^{-1} D_L, so P^{-1} K = P^{-1} D_L H = M H
    PK = Mmat @ s.H().toarray()
    A = s.A().toarray(); Bt = s.B.T.toarray(); Hp = s.H_p().toarray()
    Xi = commutator(s).toarray()
    Hp_inv_Xi = np.linalg.solve(Hp, Xi)
    nu = s.nu_total
    top_left = np.eye(nu) - np.linalg.solve(A, Bt @ Hp_inv_Xi)
    np.testing.assert_allclose(PK[:nu, :nu], top_left, atol=1e-10)
    np.testing.assert_allclose(PK[:nu, nu:], 0.0, atol=1e-10)
    np.testing.assert_allclose(PK[nu:, :nu], Hp_inv_Xi, atol=1e-10)
    np.testing.assert_allclose(PK[nu:, nu:], np.eye(s.ncell), atol=1e-10)


@pytest.mark.parametrize("n", [(32, 24), (8, 8, 6)])
def test_constant_medium_exact_blocks_one_iteration(n):
    """Constant rho, mu, lambda, gamma: Xi = 0, so P = K and the
    preconditioned system is the identity -- FGMRES converges in one
    iteration (with a lucky Arnoldi breakdown)."""
    vp, vs, rho = W.constant_medium(n, 2.0, 1.0, 1.0)
    s = ElasticSystem(n, (1.0,) * len(n), vp, vs, rho, omega=0.6, abc_width=0)
    M = BlockAcoustic(s, alpha=0.0, solver="exact")
    b = np.zeros(s.ndof, dtype=np.complex128)
    b[s.face_sizes[0] + s.face_sizes[1] // 2] = -1.0
    H = s.H()
    res = fgmres(lambda x: H @ x, M, b, restart=20, tol=1e-10, maxit=50)
    assert res.iters == 1
    assert res.relres_true < 1e-10


def _linear_problem(n1, n2, omega, lam_factor):
    n = (n1, n2)
    h = (16.0 / n1, 5.0 / n2)
    vp, vs, rho = W.linear_medium(n, lam_factor=lam_factor)
    s = ElasticSystem(n, h, vp, vs, rho, omega=omega, abc_width=20,
                      abc_sides=W.abc_all_but_top(2))
    b = W.point_source_rhs(n, h, [(1, (n1 // 2, 1))])[0]
    return s, b


@pytest.mark.slow
@pytest.mark.parametrize("row", [0, 1])
def test_table_scalability_linear(row):
    """Non-restarted GMRES with exactly solved blocks on the paper's linear
    media reproduces Table scalability_linear within one iteration."""
    g = json.load(open(os.path.join(GOLD, "tab_scalability_linear.json")))
    r = g["rows"][row]
    for lf, expect in zip(g["columns"], r["iters"]):
        s, b = _linear_problem(*r["grid"], r["omega_over_pi"] * math.pi, lf)
        M = BlockAcoustic(s, alpha=0.0, solver="exact")
        H = s.H()
        res = fgmres(lambda x: H @ x, M, b, restart=1000, tol=1e-6, maxit=200)
        assert res.relres_true < 1e-6
        assert abs(res.iters - expect) <= 1, (r["grid"], lf, res.iters, expect)


@pytest.mark.slow
def test_table_2Dlinear_block_acoustic_wcycle():
    """GMRES(5) with one W(1,2) damped-Jacobi cycle per block on the linear
    media at 400 x 128, 2/3/4 levels, reproduces the block-acoustic columns
    of Table 2Dlinear within 10%."""
    g = json.load(open(os.path.join(GOLD, "tab_2Dlinear.json")))
    r = g["rows"][0]
    s, b = _linear_problem(*r["grid"], r["omega_over_pi"] * math.pi, 1.0)
    H = s.H()
    for L, a, expect in zip(r["levels"], r["alpha"], r["iters"]):
        M = BlockAcoustic(s, alpha=a, solver="mg", levels=L, cycle="W",
                          nu=(1, 2), damping=(0.8, 0.8, 0.3))
        res = fgmres(lambda x: H @ x, M, b, restart=5, tol=1e-6, maxit=500)
        assert res.relres_true < 1e-6
        assert abs(res.iters - expect) <= 0.1 * expect, (L, res.iters, expect)


def test_tilde_Ap_symmetric_and_equal_to_Ap_for_constant_mu():
    """The alternative of the Remark after eq. prec, A~_p = B A_f(mu) B^T -
    w^2 M_p, puts the weighting between divergence and gradient: it is
    complex symmetric (A_p = B B^T diag(mu) - w^2 M_p is not, for varying mu),
    and for constant mu the two coincide, boundary cells included."""
    s = hetero((12, 10), 5)
    At = s.A_p_tilde().toarray()
    assert np.abs(At - At.T).max() <= 1e-13 * np.abs(At).max()
    A = s.A_p().toarray()
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()
    rng = np.random.default_rng(6)
    shape = (8, 10)
    rho = rng.uniform(1.0, 2.0, shape)
    vs = np.sqrt(1.5 / rho)                 # mu = rho vs^2 = 1.5 everywhere
    vp = vs * rng.uniform(1.8, 2.2, shape)
    c = ElasticSystem((10, 8), (1.0, 1.1), vp, vs, rho, omega=0.9, abc_width=2,
                      abc_sides=W.ABC_ALL[2])
    np.testing.assert_allclose(c.A_p_tilde().toarray(), c.A_p().toarray(), rtol=0, atol=1e-12)


def test_tilde_Ap_equivalent_on_smooth_medium():
    """Remark after eq. prec: on a smooth medium A~_p and A_p give equivalent
    methods -- with exact block solves, FGMRES needs the same number of
    iterations (within one) with either distributor and H_p."""
    n = (32, 32)
    y = np.linspace(0.0, 1.0, n[1])[:, None] * np.ones((1, n[0]))
    vp = 2.0 + y
    vs = 0.5 * vp
    rho = np.ones_like(vp)
    om = W.omega_for_ppw(vs, (1.0, 1.0), 10.0)
    s = ElasticSystem(n, (1.0, 1.0), vp, vs, rho, om, 6, W.abc_all_but_top(2))
    H = s.H()
    b = W.point_source_rhs(n, (1.0, 1.0), [(1, (n[0] // 2, 1))])[0]
    its = []
    for tilde in (False, True):
        M = BlockAcoustic(s, alpha=0.0, solver="exact", tilde_Ap=tilde)
        its.append(fgmres(lambda v: H @ v, M, b, restart=30, tol=1e-6, maxit=200).iters)
    assert abs(its[0] - its[1]) <= 1, its


def test_power_method_matches_dense_spectral_radius():
    """The matrix-free power method on Z(alpha) (LU solves for the shifted
    blocks) converges to the spectral radius of the dense Z(alpha) on a tiny
    heterogeneous grid; alpha = 0 is eq. Z of Theorem 3.1."""
    from oracle.analysis import ZOperator, power_method
    s = hetero((10, 8), 7, omega=1.0)
    rng = np.random.default_rng(8)
    v0 = rng.standard_normal(s.ncell) + 1j * rng.standard_normal(s.ncell)
    for alpha in (0.0, 0.3):
        rho = np.abs(np.linalg.eigvals(Z_matrix(s, alpha))).max()
        op = ZOperator(s, alpha)
        v = rng.standard_normal(s.ncell) + 1j * rng.standard_normal(s.ncell)
        np.testing.assert_allclose(op(v), Z_matrix(s, alpha) @ v, rtol=1e-10, atol=1e-12 * np.linalg.norm(v))
        est = power_method(op, v0, 300)
        assert abs(est[-1] - rho) <= 2e-3 * rho, (alpha, est[-1], rho)


def test_Z_vanishes_for_constant_media_and_shrinks_with_the_shift():
    """Constant media: Xi = 0, so Z = 0 (one-iteration convergence).  On a
    heterogeneous grid the spectral radius of Z(alpha) decreases as the
    shift grows (Section 5, the rho(Z) curves)."""
    n = (10, 8)
    vp, vs, rho = W.constant_medium(n, 2.0, 1.0, 1.0)
    c = ElasticSystem(n, (1.0, 1.0), vp, vs, rho, omega=1.0, abc_width=0, abc_sides=0)
    assert np.abs(Z_matrix(c)).max() <= 1e-10
    s = hetero((12, 10), 9, omega=1.5)
    radii = [np.abs(np.linalg.eigvals(Z_matrix(s, a))).max() for a in (0.0, 0.2, 0.5, 1.0)]
    assert all(b < a for a, b in zip(radii, radii[1:])), radii
