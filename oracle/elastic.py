"""Oracle: MAC discretisation of the mixed elastic Helmholtz system.

Test infrastructure only (see the package docstring).

Continuous problem (Section 2.1, eq. mixed-continuous): with the pressure
p = -(lambda + mu) div u,

    [ -div mu grad - rho w^2 (1 - i gamma/w)    grad          ] [u]   [-q]
    [ -div                                      -1/(lambda+mu) ] [p] = [ 0]

Discrete system (eq. mixed-discretized): H = [A B^T; B -C] with
A = grad_h^T A_e(mu) grad_h - w^2 M, B^T = grad_h, B = -div_h,
C = diag(1/(lambda + mu)), M = A_f(rho (1 - i gamma/w)).  A is block diagonal
with one acoustic operator A_k per displacement component.

Layout.  u_k lives on the k-faces, p and the medium at cell centres
(Section 2.1, Figure cell).  A field is a flat array in C order of its shape
with the x axis fastest, so operators along axis a are Kronecker products
kron(..., op_a, ...) with axis 0 (x) last.  A full vector is
[u_1 | ... | u_d | p].

Readings where the paper is silent:
* boundary: every face, boundary faces included, is an unknown; differences
  that reach outside the domain use zero ghost values (u = 0 for the
  derivatives of u across the boundary, p = 0 for B^T p at boundary faces).
* A_e and A_f are arithmetic means over the cells that exist next to an
  edge (node in 2D) or face.
* absorbing layer: gamma = gamma0 + w * sum_a l_a^2 with
  l_a = max(0, W - d_a) / W and d_a the distance (in cells, cell centre to
  side) to the nearest absorbing side along axis a.
* the complex shift of eq. shift is extra attenuation: gamma/w -> gamma/w +
  alpha in the mass term of a shifted block only.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# medium

def lame_from_velocities(vp, vs, rho):
    """mu = rho vs^2 and lambda + mu = rho (vp^2 - vs^2), from
    Vp = sqrt((lambda + 2 mu)/rho) and Vs = sqrt(mu/rho) (Section 2.1)."""
    vp = np.asarray(vp, dtype=np.float64)
    vs = np.asarray(vs, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    mu = rho * vs * vs
    lam_mu = rho * (vp * vp - vs * vs)
    return mu, lam_mu


def abc_gamma(n, omega, width, sides, gamma0=0.01 * math.pi):
    """Attenuation per cell: the natural gamma0 everywhere plus a layer of
    gradually increasing attenuation of `width` cells along the absorbing
    sides (Section 4).  `sides` is a bitmask: bit 2a = low side of axis a,
    bit 2a+1 = high side.  Returns an array of the cell shape."""
    dim = len(n)
    shape = tuple(reversed(n))
    g = np.full(shape, float(gamma0))
    if width <= 0:
        return g
    for a in range(dim):
        i = np.arange(n[a], dtype=np.float64)
        d = np.full(n[a], np.inf)
        if sides & (1 << (2 * a)):
            d = np.minimum(d, i + 0.5)
        if sides & (1 << (2 * a + 1)):
            d = np.minimum(d, n[a] - i - 0.5)
        ell = np.maximum(0.0, width - d) / width
        bshape = [1] * dim
        bshape[dim - 1 - a] = n[a]
        g = g + omega * (ell ** 2).reshape(bshape)
    return g


# ----------------------------------------------------------------------------
# 1D building blocks

def diff_1d(n, h):
    """D_n: n x (n+1), (D v)_i = (v_{i+1} - v_i)/h  (nodes -> cells)."""
    e = np.ones(n)
    return sp.diags([-e, e], [0, 1], shape=(n, n + 1), format="csr") / h


def node_sum_1d(n):
    """(n+1) x n 0/1 matrix: node k sums the cells k-1 and k that exist."""
    e = np.ones(n)
    return sp.diags([e, e], [0, -1], shape=(n + 1, n), format="csr")


def kron_axes(ops):
    """Operator acting as ops[a] along axis a (x first) on C-ordered arrays
    with x fastest: kron(ops[d-1], ..., ops[1], ops[0])."""
    out = ops[-1]
    for op in reversed(ops[:-1]):
        out = sp.kron(out, op, format="csr")
    return sp.csr_matrix(out)


def eye(n):
    return sp.identity(n, format="csr")


def loc_shape(n, nodal):
    """Shape (slowest first) of a location with the given nodal axes."""
    return tuple(reversed([n[a] + (1 if nodal[a] else 0) for a in range(len(n))]))


def average_from_cells(n, nodal, cell_values):
    """Arithmetic mean over the existing adjacent cells, from cell centres to
    the location whose axes in `nodal` are nodal (faces, edges, nodes)."""
    ops = [node_sum_1d(n[a]) if nodal[a] else eye(n[a]) for a in range(len(n))]
    S = kron_axes(ops)
    v = np.asarray(cell_values).ravel()
    cnt = S @ np.ones(v.shape[0])
    return (S @ v) / cnt


def face_nodal(dim, k):
    return tuple(a == k for a in range(dim))


def edge_nodal(dim, k, a):
    return tuple((b == k) or (b == a) for b in range(dim))


def derivative(n, h, nodal_from, a):
    """Derivative along axis a from a location (given by its nodal axes) to
    the location with axis a toggled.  Nodal -> cell-centred uses D_n;
    cell-centred -> nodal uses -D_n^T (zero ghosts outside the domain)."""
    ops = []
    for b in range(len(n)):
        size_b = n[b] + (1 if nodal_from[b] else 0)
        if b != a:
            ops.append(eye(size_b))
        elif nodal_from[a]:
            ops.append(diff_1d(n[a], h[a]))
        else:
            ops.append(-diff_1d(n[a], h[a]).T.tocsr())
    return kron_axes(ops)


# ----------------------------------------------------------------------------
# the system

class ElasticSystem:
    """Assembled sparse operators of the mixed elastic Helmholtz system.

    Parameters: n (cells per axis, x first), h (cell sizes), vp, vs, rho
    (cell arrays of shape reversed(n)), omega, abc_width, abc_sides,
    gamma0.  Alternatively mu / lam_mu may be given directly.
    """

    def __init__(self, n, h, vp=None, vs=None, rho=None, omega=1.0,
                 abc_width=0, abc_sides=0, gamma0=0.01 * math.pi,
                 mu=None, lam_mu=None, gamma=None):
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        self.dim = len(self.n)
        self.omega = float(omega)
        if mu is None:
            mu, lam_mu = lame_from_velocities(vp, vs, rho)
        self.mu = np.asarray(mu, dtype=np.float64).ravel()
        self.lam_mu = np.asarray(lam_mu, dtype=np.float64).ravel()
        self.rho = np.asarray(rho, dtype=np.float64).ravel()
        if gamma is None:
            gamma = abc_gamma(self.n, self.omega, abc_width, abc_sides, gamma0)
        self.gamma = np.asarray(gamma, dtype=np.float64).ravel()
        d = self.dim
        self.ncell = int(np.prod(self.n))
        self.face_shapes = [loc_shape(self.n, face_nodal(d, k)) for k in range(d)]
        self.face_sizes = [int(np.prod(s)) for s in self.face_shapes]
        self.nu_total = sum(self.face_sizes)
        self.ndof = self.nu_total + self.ncell
        # B^T = grad_h: cells -> k-faces (zero ghost p outside)
        cell = tuple(False for _ in range(d))
        self.Bt = [derivative(self.n, self.h, cell, k) for k in range(d)]
        self.B = sp.hstack([bt.T for bt in self.Bt], format="csr")
        self.C = sp.diags(1.0 / self.lam_mu, format="csr")

    # -- coefficients -------------------------------------------------------
    def mass_cells(self, alpha=0.0):
        """rho (1 - i (gamma/w + alpha)) at the cell centres."""
        return self.rho * (1.0 - 1j * (self.gamma / self.omega + alpha))

    def stiffness_A(self, k):
        """grad_h^T A_e(mu) grad_h restricted to u_k: sum over axes a of
        G_a^T diag(mu at the G_a location) G_a (real, symmetric)."""
        d = self.dim
        fn = face_nodal(d, k)
        out = None
        for a in range(d):
            G = derivative(self.n, self.h, fn, a)
            if a == k:
                mloc = self.mu          # d/dx_k of u_k lands on cell centres
            else:
                mloc = average_from_cells(self.n, edge_nodal(d, k, a), self.mu)
            term = (G.T @ sp.diags(mloc) @ G).tocsr()
            out = term if out is None else out + term
        return out.tocsr()

    def A_block(self, k, alpha=0.0):
        """Acoustic block A_k (shear velocity) on the k-faces; alpha > 0 gives
        the shifted block of eq. shift."""
        mf = average_from_cells(self.n, face_nodal(self.dim, k),
                                self.mass_cells(alpha))
        return (self.stiffness_A(k).astype(np.complex128)
                - self.omega ** 2 * sp.diags(mf)).tocsr()

    def A(self, alpha=0.0):
        return sp.block_diag([self.A_block(k, alpha) for k in range(self.dim)],
                             format="csr")

    def BBt(self):
        return (self.B @ self.B.T).tocsr()

    def A_p(self, alpha=0.0):
        """A_p = B B^T diag(mu) - w^2 M_p, M_p = diag(rho (1 - i gamma/w))
        (eq. Ap): shear-velocity acoustic operator on the cells, mu on the
        right of the Laplacian."""
        return (self.BBt() @ sp.diags(self.mu)
                - self.omega ** 2 * sp.diags(self.mass_cells(alpha))).tocsr()

    def A_p_tilde(self, alpha=0.0):
        """The alternative B A_f(mu) B^T - w^2 M_p of the Remark after
        eq. prec (mu between divergence and gradient)."""
        mu_f = [average_from_cells(self.n, face_nodal(self.dim, k), self.mu)
                for k in range(self.dim)]
        D = sp.diags(np.concatenate(mu_f))
        return (self.B @ D @ self.B.T
                - self.omega ** 2 * sp.diags(self.mass_cells(alpha))).tocsr()

    def H_p(self, alpha=0.0):
        """H_p = B B^T + A_p C (eq. Hp): pressure-velocity acoustic operator
        on the cells.  Shifted: A_p carries the extra attenuation alpha."""
        return (self.BBt() + self.A_p(alpha) @ self.C).tocsr()

    def H(self):
        """The mixed system matrix [A B^T; B -C] (eq. mixed-discretized)."""
        return sp.bmat([[self.A(), self.B.T], [self.B, -self.C]],
                       format="csr")

    # -- vector helpers -----------------------------------------------------
    def split(self, x):
        """Views [u_1, ..., u_d, p] of a flat vector."""
        out, o = [], 0
        for s in self.face_sizes + [self.ncell]:
            out.append(x[o:o + s])
            o += s
        return out

    def apply_H(self, x):
        """y = H x without forming H: A_k u_k + B_k^T p and B u - C p."""
        parts = self.split(x)
        u, p = parts[:-1], parts[-1]
        ys = []
        for k in range(self.dim):
            ys.append(self._Ak_cached(k) @ u[k] + self.Bt[k] @ p)
        yp = self.B @ np.concatenate(u) - p / self.lam_mu
        return np.concatenate(ys + [yp])

    def _Ak_cached(self, k):
        if not hasattr(self, "_Ak"):
            self._Ak = [self.A_block(k2) for k2 in range(self.dim)]
        return self._Ak[k]


# ----------------------------------------------------------------------------
# the same operator by array differences (large grids)

def _along(v, a, dim):
    """numpy axis of grid axis a (x = 0) for arrays stored slowest first."""
    return dim - 1 - a


def _diff_to_cells(v, a, h, dim):
    """(v_{i+1} - v_i)/h along axis a: nodes -> cells (the 1D D_n)."""
    ax = _along(v, a, dim)
    return np.diff(v, axis=ax) / h


def _diff_to_nodes(w, a, h, dim):
    """(w_j - w_{j-1})/h along axis a with w = 0 outside: cells -> nodes
    (the 1D -D_n^T)."""
    ax = _along(w, a, dim)
    pad = [(0, 0)] * w.ndim
    pad[ax] = (1, 1)
    return np.diff(np.pad(w, pad), axis=ax) / h


def _mean_to(v, nodal, dim):
    """Arithmetic mean over the existing adjacent cells, from cell values v
    to the location nodal along the axes in `nodal`."""
    s = v
    cnt = np.ones(v.shape)
    for a in range(dim):
        if not nodal[a]:
            continue
        ax = _along(v, a, dim)
        pad = [(0, 0)] * v.ndim
        pad[ax] = (1, 1)
        sp_, cp_ = np.pad(s, pad), np.pad(cnt, pad)
        lo = [slice(None)] * v.ndim
        hi = [slice(None)] * v.ndim
        lo[ax], hi[ax] = slice(0, -1), slice(1, None)
        s = sp_[tuple(lo)] + sp_[tuple(hi)]
        cnt = cp_[tuple(lo)] + cp_[tuple(hi)]
    return s / cnt


def apply_H_stencil(n, h, mu, lam_mu, mass, omega, x):
    """y = H x for the system of eq. mixed-discretized, evaluated field by
    field with array differences instead of an assembled matrix (for grids
    where assembling H is too slow).  mu, lam_mu (= lambda + mu) and mass
    (= rho (1 - i gamma/w)) are cell arrays of shape reversed(n); x is one
    flat vector [u_1 | ... | u_d | p].  Same readings as ElasticSystem:

      A_k u_k = sum_a G_a^T diag(mu at G_a's location) G_a u_k
                - w^2 A_f(mass) u_k,
      G_a = D along a for a = k (to the cells, mu at the cells),
      G_a = -D^T along a otherwise (to the edges / nodes nodal along k and
      a, mu averaged over the existing cells there), zero ghosts;
      y_k = A_k u_k + grad_k p,  y_p = -div u - p / (lambda + mu).
    """
    n = tuple(int(v) for v in n)
    d = len(n)
    cell = tuple(reversed(n))
    mu = np.asarray(mu, dtype=np.float64).reshape(cell)
    lam_mu = np.asarray(lam_mu, dtype=np.float64).reshape(cell)
    mass = np.asarray(mass, dtype=np.complex128).reshape(cell)
    x = np.asarray(x, dtype=np.complex128)
    shapes = [loc_shape(n, face_nodal(d, k)) for k in range(d)] + [cell]
    parts, o = [], 0
    for s in shapes:
        size = int(np.prod(s))
        parts.append(x[o:o + size].reshape(s))
        o += size
    if o != x.shape[0]:
        raise ValueError("vector length does not match the grid")
    u, p = parts[:-1], parts[-1]
    out = []
    div = np.zeros(cell, dtype=np.complex128)
    for k in range(d):
        acc = np.zeros(shapes[k], dtype=np.complex128)
        for a in range(d):
            if a == k:
                g = _diff_to_cells(u[k], a, h[a], d) * mu
                acc -= _diff_to_nodes(g, a, h[a], d)          # D^T = -(-D^T)
            else:
                g = _diff_to_nodes(u[k], a, h[a], d) * _mean_to(mu, edge_nodal(d, k, a), d)
                acc -= _diff_to_cells(g, a, h[a], d)          # (-D^T)^T = -D
        acc -= omega ** 2 * _mean_to(mass, face_nodal(d, k), d) * u[k]
        acc += _diff_to_nodes(p, k, h[k], d)                   # B_k^T p = grad_k p
        out.append(acc.ravel())
        div += _diff_to_cells(u[k], k, h[k], d)
    out.append((-div - p / lam_mu).ravel())
    return np.concatenate(out)


def medium_arrays(n, h, vp, vs, rho, omega, abc_width, abc_sides, gamma0=0.01 * math.pi):
    """(mu, lambda + mu, rho (1 - i gamma/w)) at the cells, the inputs of
    apply_H_stencil, from the velocities and the absorbing layer."""
    mu, lam_mu = lame_from_velocities(vp, vs, rho)
    gamma = abc_gamma(tuple(int(v) for v in n), omega, abc_width, abc_sides, gamma0)
    mass = np.asarray(rho, dtype=np.float64) * (1.0 - 1j * gamma / omega)
    return mu, lam_mu, mass
