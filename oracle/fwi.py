"""Oracle: least-squares misfit and its gradient with respect to per-cell
vp, vs and rho.

Test infrastructure only (see the package docstring).

The paper presents its solver as the forward solver of frequency-domain
elastic full-waveform inversion (Section 4).  For sources b_s, solutions
H(m) u_s = b_s and receivers that sample u at given dofs (P_r),

    Phi(m) = 1/2 sum_s || P_r u_s - d_s ||^2 ,
    dPhi/dm = - Re sum_s lambda_s^H (dH/dm) u_s ,
    H^H lambda_s = P_r^T (P_r u_s - d_s).

H is complex symmetric, so lambda_s = conj(H^{-1} conj(g_s)).  dH/dm comes
from the assembly of H in ``elastic``: mu enters the stiffness of every A_k
at cell centres and, through the arithmetic means, at edges; rho enters the
face mass A_f(rho (1 - i gamma/w)); lambda + mu enters C.  gamma and w are
held fixed.  Chain rule: mu = rho vs^2, lambda + mu = rho (vp^2 - vs^2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .elastic import (ElasticSystem, derivative, edge_nodal, face_nodal,
                      kron_axes, eye, node_sum_1d)


def _sum_matrix(n, nodal):
    return kron_axes([node_sum_1d(n[a]) if nodal[a] else eye(n[a])
                      for a in range(len(n))])


def dH_terms(sys: ElasticSystem, lam, u):
    """Per-cell sums T_x(c) = sum_s lam_s^H (dH/dx_c) u_s for x in
    (mu, lambda+mu, rho).  lam, u: arrays (nrhs, ndof).  Complex arrays."""
    lam = np.atleast_2d(lam)
    u = np.atleast_2d(u)
    n, d = sys.n, sys.dim
    T_mu = np.zeros(sys.ncell, dtype=np.complex128)
    T_lm = np.zeros(sys.ncell, dtype=np.complex128)
    T_rho = np.zeros(sys.ncell, dtype=np.complex128)
    for s in range(u.shape[0]):
        lp = sys.split(lam[s])
        up = sys.split(u[s])
        for k in range(d):
            fn = face_nodal(d, k)
            for a in range(d):
                G = derivative(n, sys.h, fn, a)
                val = np.conj(G @ lp[k]) * (G @ up[k])
                if a == k:
                    T_mu += val
                else:
                    S = _sum_matrix(n, edge_nodal(d, k, a))
                    cnt = S @ np.ones(sys.ncell)
                    T_mu += S.T @ (val / cnt)
            S = _sum_matrix(n, fn)
            cnt = S @ np.ones(sys.ncell)
            fval = np.conj(lp[k]) * up[k] / cnt
            T_rho += (-sys.omega ** 2) * (1.0 - 1j * sys.gamma / sys.omega) * (S.T @ fval)
        T_lm += np.conj(lp[-1]) * up[-1] / sys.lam_mu ** 2
    return T_mu, T_lm, T_rho


def chain_to_velocities(G_mu, G_lm, G_rho_direct, vp, vs, rho):
    """Gradients with respect to (vp, vs, rho) from those with respect to
    (mu, lambda+mu, rho at fixed Lame)."""
    vp, vs, rho = (np.asarray(v, dtype=np.float64).ravel() for v in (vp, vs, rho))
    g_vp = G_lm * 2.0 * rho * vp
    g_vs = G_mu * 2.0 * rho * vs - G_lm * 2.0 * rho * vs
    g_rho = G_mu * vs * vs + G_lm * (vp * vp - vs * vs) + G_rho_direct
    return g_vp, g_vs, g_rho


def misfit(sys: ElasticSystem, b, rec, d_obs, lu=None):
    """Phi and the forward fields, with direct solves."""
    if lu is None:
        lu = spla.splu(sys.H().tocsc())
    b = np.atleast_2d(b)
    U = np.stack([lu.solve(bs) for bs in b])
    res = U[:, rec] - d_obs
    return 0.5 * float(np.sum(np.abs(res) ** 2)), U, res, lu


def gradient(n, h, vp, vs, rho, omega, abc_width, abc_sides, b, rec, d_obs,
             gamma0=0.01 * np.pi, gamma=None):
    """Phi and (g_vp, g_vs, g_rho) per cell (flat), with direct solves."""
    sys = ElasticSystem(n, h, vp, vs, rho, omega, abc_width, abc_sides,
                        gamma0, gamma=gamma)
    phi, U, res, lu = misfit(sys, b, rec, d_obs)
    lam = np.zeros_like(U)
    for s in range(U.shape[0]):
        g = np.zeros(sys.ndof, dtype=np.complex128)
        np.add.at(g, rec, res[s])
        lam[s] = np.conj(lu.solve(np.conj(g)))
    T_mu, T_lm, T_rho = dH_terms(sys, lam, U)
    G_mu, G_lm, G_rho = -T_mu.real, -T_lm.real, -T_rho.real
    return phi, chain_to_velocities(G_mu, G_lm, G_rho, vp, vs, rho), U, lam
