"""Pins of the oracle's discretisation (CPU only).

Each test checks the oracle against something it does not compute itself:
the exact algebraic structure of eq. mixed-discretized (complex symmetry,
stencil widths), the vanishing commutator for constant media (footnote to
eq. vecId and the homogeneous-media remark of Section 4), a continuous
manufactured solution (second-order convergence of the MAC scheme) and a
brute-force dense inverse.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle.elastic import ElasticSystem, abc_gamma, lame_from_velocities
from oracle.analysis import commutator


def random_medium(n, seed=0):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    vp = rng.uniform(2.0, 4.0, shape)
    vs = vp * rng.uniform(0.3, 0.55, shape)
    rho = rng.uniform(1.0, 2.5, shape)
    return vp, vs, rho


@pytest.mark.parametrize("n", [(6, 5), (4, 3, 5)])
def test_lame_relations(n):
    vp, vs, rho = random_medium(n)
    mu, lm = lame_from_velocities(vp, vs, rho)
    lam = lm - mu
    np.testing.assert_allclose(np.sqrt((lam + 2 * mu) / rho), vp, rtol=1e-14)
    np.testing.assert_allclose(np.sqrt(mu / rho), vs, rtol=1e-14)


@pytest.mark.parametrize("n", [(7, 6), (5, 4, 3)])
def test_complex_symmetry(n):
    """H = H^T and A_k = A_k^T exactly (eq. mixed-discretized), and
    H_p diag(1/w) is symmetric with w = (lambda+2mu)/(lambda+mu) (eq. Hp)."""
    vp, vs, rho = random_medium(n, 1)
    s = ElasticSystem(n, (1.0,) * len(n), vp, vs, rho, omega=0.9,
                      abc_width=2, abc_sides=W.ABC_ALL[len(n)])
    H = s.H()
    assert abs(H - H.T).max() == 0.0
    for k in range(len(n)):
        Ak = s.A_block(k, alpha=0.3)
        assert abs(Ak - Ak.T).max() == 0.0
    mu, lm = lame_from_velocities(vp, vs, rho)
    w = ((lm + mu) / lm).ravel()
    S = s.H_p(alpha=0.2) @ np.diag(1.0 / w)
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    # H is not Hermitian (attenuation makes the mass complex)
    assert abs(H - H.conj().T).max() > 0


def test_stencil_widths():
    """Interior rows: A_k, H_p and A_p are 5-diagonal, B has 4 nonzeros per
    row in 2D (two 2-diagonal matrices) -- Section 4.4.2."""
    n = (8, 8)
    vp, vs, rho = random_medium(n, 2)
    s = ElasticSystem(n, (1.0, 1.0), vp, vs, rho, omega=1.0)
    nnz = lambda M: np.diff(M.tocsr().indptr)
    for k in range(2):
        assert nnz(s.A_block(k)).max() == 5
    assert nnz(s.H_p()).max() == 5
    assert nnz(s.A_p()).max() == 5
    assert nnz(s.B).max() == 4 and nnz(s.B).min() == 4
    # 3D: 7-point blocks, 6 nonzeros per row of B
    n3 = (4, 4, 4)
    vp, vs, rho = random_medium(n3, 3)
    s3 = ElasticSystem(n3, (1.0,) * 3, vp, vs, rho, omega=1.0)
    assert nnz(s3.A_block(0)).max() == 7
    assert nnz(s3.H_p()).max() == 7
    assert nnz(s3.B).min() == 6


@pytest.mark.parametrize("n", [(10, 8), (6, 4, 5)])
def test_commutator_vanishes_for_constant_media(n):
    """With constant rho, mu, lambda and gamma the MAC operators commute:
    Xi = B A - A_p B = 0, boundaries included (footnote to eq. vecId and the
    homogeneous media of Section 4).  A dropped or misplaced term in A_k,
    B or A_p breaks this."""
    vp, vs, rho = W.constant_medium(n, 3.0, 1.2, 1.7)
    s = ElasticSystem(n, tuple(0.5 + 0.25 * a for a in range(len(n))),
                      vp, vs, rho, omega=1.3, abc_width=0)
    Xi = commutator(s)
    scale = abs(s.B @ s.A()).max()
    assert abs(Xi).max() <= 1e-12 * scale
    # and with a heterogeneous medium it does not vanish
    vp, vs, rho = random_medium(n, 4)
    s2 = ElasticSystem(n, (1.0,) * len(n), vp, vs, rho, omega=1.3)
    assert abs(commutator(s2)).max() > 1e-3


def test_abc_profile():
    """Layer of gradually increasing attenuation on the absorbing sides only
    (Section 4): gamma0 inside, growing towards the sides, none on top."""
    n, W_, om = (40, 30), 10, 2.0
    g = abc_gamma(n, om, W_, W.abc_all_but_top(2), gamma0=0.01 * math.pi)
    assert g.shape == (30, 40)
    g0 = 0.01 * math.pi
    assert np.allclose(g[5:20, 12:28], g0)                 # interior
    assert np.allclose(g[0:5, 12:28], g0)                  # top: no layer
    assert np.all(np.diff(g[15, :11]) < 0)                 # left side grows outwards
    assert np.all(np.diff(g[15, 29:]) > 0)                 # right side
    assert np.all(np.diff(g[20:, 20]) > 0)                 # bottom
    assert g[15, 0] == pytest.approx(g0 + om * ((W_ - 0.5) / W_) ** 2)
    assert g[29, 0] == pytest.approx(g0 + 2 * om * ((W_ - 0.5) / W_) ** 2)


def _manufactured(nc):
    """Discrete solve of the mixed system against a smooth exact solution of
    the continuous problem (eq. mixed-continuous) on [0,1]^2 with smooth
    variable coefficients; returns the max face error of u."""
    import sympy as sym
    x, y = sym.symbols("x y")
    mu = 1 + sym.Rational(1, 2) * sym.sin(2 * sym.pi * x) * sym.cos(sym.pi * y)
    lm = 3 + sym.cos(sym.pi * x * y)                       # lambda + mu
    rho = 1 + sym.Rational(3, 10) * x * y
    gam = sym.Rational(1, 10) + sym.Rational(1, 5) * x
    om = 2
    b = (sym.sin(sym.pi * x) * sym.sin(sym.pi * y)) ** 4
    u1 = b * sym.cos(sym.pi * y)
    u2 = b * (1 + x)
    p = -lm * (sym.diff(u1, x) + sym.diff(u2, y))
    m = rho * (1 - sym.I * gam / om)

    def lap_mu(u):
        return sym.diff(mu * sym.diff(u, x), x) + sym.diff(mu * sym.diff(u, y), y)
    f1 = -lap_mu(u1) - om ** 2 * m * u1 + sym.diff(p, x)
    f2 = -lap_mu(u2) - om ** 2 * m * u2 + sym.diff(p, y)
    F = [sym.lambdify((x, y), e, "numpy") for e in (mu, lm, rho, gam, u1, u2, f1, f2)]
    h = 1.0 / nc
    xc = (np.arange(nc) + 0.5) * h
    xn = np.arange(nc + 1) * h
    Xc, Yc = np.meshgrid(xc, xc)                 # (n2, n1) cells
    mu_c = F[0](Xc, Yc); lm_c = F[1](Xc, Yc); rho_c = F[2](Xc, Yc); g_c = F[3](Xc, Yc)
    vs = np.sqrt(mu_c / rho_c)
    vp = np.sqrt((lm_c + mu_c) / rho_c)          # (lambda + 2 mu) / rho
    s = ElasticSystem((nc, nc), (h, h), vp, vs, rho_c, omega=om,
                      gamma=g_c.ravel())
    X1, Y1 = np.meshgrid(xn, xc)                 # u1 faces (n2, n1+1)
    X2, Y2 = np.meshgrid(xc, xn)                 # u2 faces (n2+1, n1)
    rhs = np.concatenate([np.broadcast_to(F[6](X1, Y1), X1.shape).ravel(),
                          np.broadcast_to(F[7](X2, Y2), X2.shape).ravel(),
                          np.zeros(nc * nc)]).astype(np.complex128)
    sol = spla.spsolve(s.H().tocsc(), rhs)
    ex = np.concatenate([F[4](X1, Y1).ravel(), F[5](X2, Y2).ravel()])
    return np.abs(sol[:s.nu_total] - ex).max()


def test_manufactured_solution_second_order():
    """The MAC scheme converges at second order to a smooth exact solution
    with variable mu, lambda, rho and gamma: errors drop ~4x per halving of
    h.  A wrong sign, transposed operand or misplaced average would stall
    the convergence or converge to the wrong limit."""
    e = [_manufactured(nc) for nc in (16, 32, 64)]
    assert e[0] / e[1] > 3.2 and e[1] / e[2] > 3.5, e
    assert e[2] < 5e-3


def test_dense_inverse_agrees_with_sparse_lu():
    """Brute force on a 16 x 16 grid (800 unknowns): the dense inverse of H
    and the sparse LU solve agree."""
    n = (16, 16)
    vp, vs, rho = random_medium(n, 5)
    s = ElasticSystem(n, (1.0, 1.0), vp, vs, rho, omega=0.7, abc_width=4,
                      abc_sides=W.ABC_ALL[2])
    H = s.H()
    assert H.shape == (800, 800)
    b = np.random.default_rng(0).standard_normal(800) + 0j
    x_dense = np.linalg.inv(H.toarray()) @ b
    x_lu = spla.splu(H.tocsc()).solve(b)
    assert np.linalg.norm(x_dense - x_lu) <= 1e-10 * np.linalg.norm(x_lu)
    assert np.linalg.norm(H @ x_lu - b) <= 1e-10 * np.linalg.norm(b)


def test_apply_H_matches_assembled():
    n = (9, 7, 5)
    vp, vs, rho = random_medium(n, 6)
    s = ElasticSystem(n, (1.0, 0.8, 1.2), vp, vs, rho, omega=1.1,
                      abc_width=2, abc_sides=W.ABC_ALL[3])
    x = np.random.default_rng(1).standard_normal(s.ndof) * (1 + 0.5j)
    np.testing.assert_allclose(s.apply_H(x), s.H() @ x, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n,h,sides", [((9, 7), (1.0, 0.8), "all"), ((6, 5, 4), (1.0, 0.8, 1.2), "top"),
                                       ((3, 8, 2), (0.5, 1.0, 1.0), "all")])
def test_array_difference_H_matches_assembly(n, h, sides):
    """The array-difference evaluation of H (large grids) equals the
    assembled H, whose entries the other pins fix, with a heterogeneous
    medium and an absorbing layer; and it is complex symmetric on its own
    (x^T H y = y^T H x), the structure of eq. mixed-discretized."""
    from oracle.elastic import apply_H_stencil, medium_arrays
    vp, vs, rho = random_medium(n, 8)
    dim = len(n)
    sd = W.ABC_ALL[dim] if sides == "all" else W.abc_all_but_top(dim)
    s = ElasticSystem(n, h, vp, vs, rho, omega=1.3, abc_width=2, abc_sides=sd)
    mu, lm, m = medium_arrays(n, h, vp, vs, rho, 1.3, 2, sd)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(s.ndof) + 1j * rng.standard_normal(s.ndof)
    y = rng.standard_normal(s.ndof) + 1j * rng.standard_normal(s.ndof)
    Hx = apply_H_stencil(n, h, mu, lm, m, 1.3, x)
    Hy = apply_H_stencil(n, h, mu, lm, m, 1.3, y)
    ref = s.H() @ x
    assert np.linalg.norm(Hx - ref) <= 1e-14 * np.linalg.norm(ref)
    assert abs(y @ Hx - x @ Hy) <= 1e-13 * np.linalg.norm(Hx) * np.linalg.norm(y)
