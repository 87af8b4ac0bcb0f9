"""Pins of the oracle's misfit gradient (CPU only): central finite
differences of the misfit computed with direct solves, and a brute-force
check of the per-cell dH/dm terms against re-assembled operators."""
import numpy as np
import pytest

import workloads as W
from oracle.elastic import ElasticSystem
from oracle.fwi import dH_terms, gradient, misfit


def _setup(n=(12, 10), seed=0):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    vp = rng.uniform(2.0, 3.0, shape)
    vs = vp * rng.uniform(0.4, 0.55, shape)
    rho = rng.uniform(1.0, 2.0, shape)
    h = (1.0, 1.0)
    src = [(1, (n[0] // 4, 1)), (1, (3 * n[0] // 4, 1))]
    rec = W.receiver_indices(n, [(1, (i, 1)) for i in range(1, n[0], 2)])
    b = W.point_source_rhs(n, h, src)
    omega, width, sides = 0.9, 3, W.abc_all_but_top(2)
    # observed data from a perturbed medium
    s_true = ElasticSystem(n, h, vp * 1.03, vs * 0.98, rho, omega, width, sides)
    _, U, _, _ = misfit(s_true, b, rec, np.zeros((2, len(rec))))
    d_obs = U[:, rec]
    return n, h, vp, vs, rho, omega, width, sides, b, rec, d_obs


def test_gradient_matches_central_differences():
    n, h, vp, vs, rho, om, wd, sd, b, rec, d = _setup()
    phi, (gvp, gvs, grho), _, _ = gradient(n, h, vp, vs, rho, om, wd, sd, b, rec, d)
    # the ABC attenuation depends on omega only, so it stays fixed
    rng = np.random.default_rng(9)
    eps = 1e-6
    for _ in range(4):
        dvp, dvs, drho = (rng.standard_normal(vp.shape) * v for v in (vp, vs, rho))

        def phi_at(t):
            s = ElasticSystem(n, h, vp + t * dvp, vs + t * dvs, rho + t * drho,
                              om, wd, sd)
            return misfit(s, b, rec, d)[0]
        fd = (phi_at(eps) - phi_at(-eps)) / (2 * eps)
        an = gvp @ dvp.ravel() + gvs @ dvs.ravel() + grho @ drho.ravel()
        assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)


def test_dH_terms_brute_force():
    """lam^H (dH/dm_c) u by re-assembling H at m_c +- eps for a few cells."""
    n, h, vp, vs, rho, om, wd, sd, *_ = _setup((6, 5), 1)
    s = ElasticSystem(n, h, vp, vs, rho, om, wd, sd)
    rng = np.random.default_rng(2)
    lam = rng.standard_normal(s.ndof) + 1j * rng.standard_normal(s.ndof)
    u = rng.standard_normal(s.ndof) + 1j * rng.standard_normal(s.ndof)
    T_mu, T_lm, T_rho = dH_terms(s, lam, u)
    eps = 1e-6
    mu = s.mu.reshape(vp.shape); lm = s.lam_mu.reshape(vp.shape)
    for c in [0, 7, 14, 29]:
        for which, T in (("mu", T_mu), ("lm", T_lm), ("rho", T_rho)):
            vals = []
            for sgn in (1, -1):
                m2, l2, r2 = mu.copy(), lm.copy(), rho.copy()
                tgt = {"mu": m2, "lm": l2, "rho": r2}[which]
                tgt.ravel()[c] += sgn * eps
                s2 = ElasticSystem(n, h, rho=r2, omega=om, mu=m2, lam_mu=l2,
                                   gamma=s.gamma)
                vals.append(np.conj(lam) @ (s2.H() @ u))
            fd = (vals[0] - vals[1]) / (2 * eps)
            assert abs(fd - T[c]) <= 1e-6 * max(1.0, abs(T[c])), (which, c)
