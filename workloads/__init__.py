"""Seeded synthetic inputs for the elastic Helmholtz solver.

This module is shared by the tests, the benchmark and the smoke check.  It
draws media (per-cell P velocity, S velocity and density), picks the angular
frequency from a points-per-wavelength rule and places point sources and
receivers.  It holds none of the solver's arithmetic: no operator, no
absorbing layer, no multigrid and no Krylov step lives here.

Arrays are cell-centred and C-contiguous with x fastest: a 2D medium has
shape (n2, n1), a 3D medium (n3, n2, n1).  Depth is the last axis (y in 2D,
z in 3D) and index 0 along it is the top of the domain.

The paper's geophysical media (Marmousi2, SEAM, SEG/EAGE salt, Overthrust)
are not available; the layered / random media below stand in for them.  They
keep the paper's structure: horizontally layered, heterogeneous, Poisson
ratio between 0.25 and 0.49, about ten points per shear wavelength and
sources near the top (Section 4 of the paper).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "constant_medium",
    "linear_medium",
    "layered_medium",
    "layered_inclusion_medium_3d",
    "omega_for_ppw",
    "vs_from_poisson",
    "config",
    "ABC_ALL",
    "abc_all_but_top",
]


def abc_all_but_top(dim: int) -> int:
    """Bitmask of absorbing sides: bit 2a is the low side of axis a, bit 2a+1
    the high side.  The top (low side of the depth axis) is left out."""
    mask = (1 << (2 * dim)) - 1
    return mask & ~(1 << (2 * (dim - 1)))


ABC_ALL = {2: 0b1111, 3: 0b111111}


@dataclass
class Workload:
    """One synthetic problem: grid, medium, frequency, sources, receivers and
    the solver settings the problem is run with."""

    name: str
    n: tuple            # cells per axis, x first
    h: tuple            # cell size per axis
    vp: np.ndarray
    vs: np.ndarray
    rho: np.ndarray
    omega: float
    abc_width: int
    abc_sides: int
    sources: list       # list of u-face positions (component, index tuple x-first)
    receivers: list = field(default_factory=list)
    levels: int = 3
    nu: tuple = (1, 2)
    damping: tuple = (0.8, 0.8, 0.3)
    alpha: float = 0.1
    restart: int = 20
    tol: float = 1e-6
    gamma0: float = 0.01 * math.pi
    intergrid: str = "full"        # "mixed": eq. tildeRu1 restriction (3D setting)

    @property
    def dim(self) -> int:
        return len(self.n)


def vs_from_poisson(vp: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """S velocity for a given P velocity and Poisson ratio sigma, from
    vp^2 / vs^2 = 2(1 - sigma) / (1 - 2 sigma)."""
    return vp * np.sqrt((1.0 - 2.0 * sigma) / (2.0 * (1.0 - sigma)))


def omega_for_ppw(vs: np.ndarray, h, ppw: float) -> float:
    """Angular frequency giving `ppw` grid points per shear wavelength where
    the shear velocity is lowest (wavelength = 2 pi vs / omega)."""
    return 2.0 * math.pi * float(np.min(vs)) / (ppw * float(max(h)))


def constant_medium(n, vp: float, vs: float, rho: float):
    shape = tuple(reversed(n))
    return (np.full(shape, float(vp)), np.full(shape, float(vs)),
            np.full(shape, float(rho)))


def linear_medium(n, rho_range=(2.0, 3.0), mu_range=(1.0, 15.0),
                  lam_range=(4.0, 20.0), lam_factor: float = 1.0):
    """Density and Lame coefficients varying linearly with depth (the
    paper's 'linear media', Section 4), returned as (vp, vs, rho).

    The coefficients are sampled at cell centres, top to bottom."""
    shape = tuple(reversed(n))
    nd = shape[0]
    t = (np.arange(nd) + 0.5) / nd
    bshape = (nd,) + (1,) * (len(n) - 1)
    rho = (rho_range[0] + t * (rho_range[1] - rho_range[0])).reshape(bshape)
    mu = (mu_range[0] + t * (mu_range[1] - mu_range[0])).reshape(bshape)
    lam = lam_factor * (lam_range[0] + t * (lam_range[1] - lam_range[0])).reshape(bshape)
    rho = np.broadcast_to(rho, shape).copy()
    mu = np.broadcast_to(mu, shape).copy()
    lam = np.broadcast_to(lam, shape).copy()
    vs = np.sqrt(mu / rho)
    vp = np.sqrt((lam + 2.0 * mu) / rho)
    return vp, vs, rho


def _smooth_field(rng, shape, corr):
    from scipy.ndimage import gaussian_filter
    g = rng.standard_normal(shape)
    g = gaussian_filter(g, sigma=corr, mode="reflect")
    g -= g.mean()
    g /= g.std()
    return g


def layered_medium(n, seed: int, n_layers: int = 8, vp_range=(1.5, 4.5),
                   sigma_range=(0.25, 0.45), pert: float = 0.05,
                   corr: float = 20.0):
    """Horizontally layered medium with a smoothed random perturbation.

    Per layer vp ~ U(vp_range) and sigma ~ U(sigma_range); a white N(0,1)
    field smoothed by a Gaussian of std `corr` cells and renormalised to unit
    std multiplies vp by (1 + pert * g).  vs follows from sigma, rho = 1."""
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    nd = shape[0]
    vp_l = rng.uniform(*vp_range, size=n_layers)
    sg_l = rng.uniform(*sigma_range, size=n_layers)
    layer = np.minimum((np.arange(nd) * n_layers) // nd, n_layers - 1)
    bshape = (nd,) + (1,) * (len(n) - 1)
    vp = np.broadcast_to(vp_l[layer].reshape(bshape), shape).copy()
    sg = np.broadcast_to(sg_l[layer].reshape(bshape), shape).copy()
    g = _smooth_field(rng, shape, corr)
    vp = vp * (1.0 + pert * g)
    vs = vs_from_poisson(vp, sg)
    rho = np.ones(shape)
    return vp, vs, rho


def layered_inclusion_medium_3d(n, seed: int, n_layers: int = 8,
                                vp_range=(1.5, 4.0), sigma_range=(0.25, 0.45),
                                std_cells: float = 16.0, amp: float = 0.2):
    """3D layered medium (layers along z) plus one Gaussian inclusion whose
    centre is uniform in the middle third of the box."""
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))      # (n3, n2, n1)
    nd = shape[0]
    vp_l = rng.uniform(*vp_range, size=n_layers)
    sg_l = rng.uniform(*sigma_range, size=n_layers)
    layer = np.minimum((np.arange(nd) * n_layers) // nd, n_layers - 1)
    vp = np.broadcast_to(vp_l[layer].reshape(nd, 1, 1), shape).copy()
    sg = np.broadcast_to(sg_l[layer].reshape(nd, 1, 1), shape).copy()
    centre = [rng.uniform(nk / 3.0, 2.0 * nk / 3.0) for nk in n]
    sign = rng.choice([-1.0, 1.0])
    z, y, x = np.meshgrid(*(np.arange(s) + 0.5 for s in shape), indexing="ij")
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    vp = vp * (1.0 + sign * amp * np.exp(-0.5 * r2 / std_cells ** 2))
    vp = np.clip(vp, *vp_range)
    vs = vs_from_poisson(vp, sg)
    rho = np.ones(shape)
    return vp, vs, rho


def config(k: int, scale: int = 1) -> Workload:
    """The five benchmark workloads.  `scale` > 1 divides every grid axis
    (for quick tests at the same structure); scale = 1 is the full size.

    1: 64^2 constant medium, centre source, 3-level V-cycle.
    2: 1024^2 layered + random medium, one top source.
    3: 512^2 layered medium, 16 top sources, 256 receivers (gradient).
    4: 2048^2 layered medium, sigma up to 0.49, 32 top sources (batched).
    5: 192^3 layered medium with a Gaussian inclusion, 4 top sources.
    """
    if k == 1:
        n = (64 // scale, 64 // scale)
        vp, vs, rho = constant_medium(n, 2.0, 1.0, 1.0)
        h = (1.0, 1.0)
        omega = omega_for_ppw(vs, h, 10.0)
        src = [(1, (n[0] // 2, n[1] // 2))]
        return Workload("config1_const_64", n, h, vp, vs, rho, omega,
                        abc_width=max(10 // scale, 1), abc_sides=ABC_ALL[2],
                        sources=src, levels=3, alpha=0.1, restart=20)
    if k == 2:
        n = (1024 // scale, 1024 // scale)
        vp, vs, rho = layered_medium(n, seed=0)
        h = (1.0, 1.0)
        omega = omega_for_ppw(vs, h, 10.0)
        src = [(1, (n[0] // 2, 1))]
        return Workload("config2_layered_1024", n, h, vp, vs, rho, omega,
                        abc_width=20, abc_sides=abc_all_but_top(2),
                        sources=src, levels=6, alpha=0.7, restart=4)
    if k == 3:
        n = (512 // scale, 512 // scale)
        vp, vs, rho = layered_medium(n, seed=1)
        h = (1.0, 1.0)
        omega = omega_for_ppw(vs, h, 10.0)
        src = [(1, ((16 + 32 * s) // scale, 1)) for s in range(16)]
        rec = [(1, ((1 + 2 * r) // scale, 1)) for r in range(256)]
        return Workload("config3_fwi_512", n, h, vp, vs, rho, omega,
                        abc_width=20, abc_sides=abc_all_but_top(2),
                        sources=src, receivers=rec, levels=5, alpha=0.7,
                        restart=4)
    if k == 4:
        n = (2048 // scale, 2048 // scale)
        vp, vs, rho = layered_medium(n, seed=3, sigma_range=(0.25, 0.49))
        h = (1.0, 1.0)
        omega = omega_for_ppw(vs, h, 10.0)
        src = [(1, ((32 + 64 * s) // scale, 1)) for s in range(32)]
        return Workload("config4_layered_2048_b32", n, h, vp, vs, rho, omega,
                        abc_width=20, abc_sides=abc_all_but_top(2),
                        sources=src, levels=7, alpha=0.7, restart=4)
    if k == 5:
        n = (192 // scale,) * 3
        vp, vs, rho = layered_inclusion_medium_3d(n, seed=4)
        h = (1.0, 1.0, 1.0)
        omega = omega_for_ppw(vs, h, 8.0)
        m = n[0]
        src = [(2, (m // 3, m // 3, 1)), (2, (2 * m // 3, m // 3, 1)),
               (2, (m // 3, 2 * m // 3, 1)), (2, (2 * m // 3, 2 * m // 3, 1))]
        return Workload("config5_layered_192cube", n, h, vp, vs, rho, omega,
                        abc_width=max(12 // scale, 1), abc_sides=abc_all_but_top(3),
                        sources=src, levels=4, nu=(2, 2),
                        damping=(0.8, 0.8, 0.2), alpha=1.2, restart=6,
                        intergrid="mixed")
    raise ValueError(f"unknown config {k}")


def field_shapes(n):
    """Array shapes (slowest axis first) of the fields u_1..u_d and p in the
    vector layout [u_1 | ... | u_d | p]: u_k lives on the k-faces (one more
    point along axis k), p at the cell centres."""
    dim = len(n)
    shapes = []
    for k in range(dim):
        m = list(n)
        m[k] += 1
        shapes.append(tuple(reversed(m)))
    shapes.append(tuple(reversed(n)))
    return shapes


def point_source_rhs(n, h, sources, dtype=np.complex128):
    """Right-hand sides (nrhs, ndof) for unit point forces.

    Each source (k, idx) is a unit force along axis k at the k-face with
    x-first index `idx`; the system's right-hand side is (-q, 0) with q the
    discrete delta 1/(h_1 ... h_d) at that face."""
    shapes = field_shapes(n)
    sizes = [int(np.prod(s)) for s in shapes]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    b = np.zeros((len(sources), int(offs[-1])), dtype=dtype)
    vol = float(np.prod(h))
    for s, (k, idx) in enumerate(sources):
        flat = np.ravel_multi_index(tuple(reversed(idx)), shapes[k])
        b[s, offs[k] + flat] = -1.0 / vol
    return b


def receiver_indices(n, receivers):
    """Flat dof indices (into [u_1 | ... | u_d | p]) of receiver positions
    (k, idx): each receiver records u_k at the k-face `idx`."""
    shapes = field_shapes(n)
    sizes = [int(np.prod(s)) for s in shapes]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    out = []
    for k, idx in receivers:
        out.append(int(offs[k] + np.ravel_multi_index(tuple(reversed(idx)), shapes[k])))
    return np.asarray(out, dtype=np.int64)
