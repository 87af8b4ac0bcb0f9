"""Pins of the oracle's FGMRES (CPU only): the flexible Arnoldi relation,
orthonormality, the minimal-residual property against a brute-force
Krylov least-squares problem, and the edge cases."""
import numpy as np
import pytest

from oracle.fgmres import fgmres


def _mat(n, seed):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.4 + 1j * rng.standard_normal((n, n)) * 0.2
    return A


def test_flexible_arnoldi_relation_and_orthonormality():
    n = 60
    A = _mat(n, 0)
    rng = np.random.default_rng(1)
    D = np.diag(rng.uniform(0.5, 2.0, n))
    calls = {"k": 0}

    def M(v):                       # a preconditioner that changes each call
        calls["k"] += 1
        return (D + 0.01 * calls["k"] * np.eye(n)) @ v
    b = rng.standard_normal(n) + 0j
    rec = {}
    fgmres(lambda x: A @ x, M, b, restart=12, tol=1e-30, maxit=12, record=rec)
    V = np.stack(rec["V"], axis=1)
    Z = np.stack(rec["Z"], axis=1)
    Hb = rec["Hbar"]
    assert V.shape[1] == Hb.shape[0] and Z.shape[1] == Hb.shape[1]
    np.testing.assert_allclose(A @ Z, V @ Hb, atol=1e-12)
    np.testing.assert_allclose(V.conj().T @ V, np.eye(V.shape[1]), atol=1e-12)


def test_minimal_residual_matches_brute_force():
    """With the identity preconditioner and no restart, the iterate after k
    steps minimises ||b - A x|| over the Krylov space K_k(A, b): compare with
    a least-squares solve on the explicit (orthogonalised) Krylov basis."""
    n, k = 40, 7
    A = _mat(n, 2)
    b = np.random.default_rng(3).standard_normal(n) + 0j
    res = fgmres(lambda x: A @ x, lambda v: v, b, restart=100, tol=1e-30, maxit=k)
    K = np.stack([np.linalg.matrix_power(A, j) @ b for j in range(k)], axis=1)
    Q, _ = np.linalg.qr(K)
    c, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    x_bf = Q @ c
    assert res.iters == k
    np.testing.assert_allclose(np.linalg.norm(b - A @ res.x),
                               np.linalg.norm(b - A @ x_bf), rtol=1e-9)
    np.testing.assert_allclose(res.history[-1], np.linalg.norm(b - A @ x_bf) / np.linalg.norm(b), rtol=1e-8)


def test_estimate_equals_true_residual_and_restart():
    n = 80
    A = _mat(n, 4)
    b = np.random.default_rng(5).standard_normal(n) + 1j
    res = fgmres(lambda x: A @ x, lambda v: v, b, restart=5, tol=1e-8, maxit=400)
    assert res.converged
    assert res.relres_true < 1e-8
    np.testing.assert_allclose(res.history[-1], res.relres_true, rtol=1e-4)


def test_zero_rhs_and_maxit():
    n = 20
    A = _mat(n, 6)
    res = fgmres(lambda x: A @ x, lambda v: v, np.zeros(n, complex), restart=5)
    assert res.iters == 0 and np.all(res.x == 0)
    b = np.ones(n, complex)
    res = fgmres(lambda x: A @ x, lambda v: v, b, restart=3, tol=1e-14, maxit=4)
    assert res.iters == 4 and not res.converged


def test_lucky_breakdown_exact_preconditioner():
    n = 30
    A = _mat(n, 7)
    Ainv = np.linalg.inv(A)
    b = np.arange(n) + 1j
    res = fgmres(lambda x: A @ x, lambda v: Ainv @ v, b, restart=10, tol=1e-12, maxit=10)
    assert res.iters == 1 and res.relres_true < 1e-12
