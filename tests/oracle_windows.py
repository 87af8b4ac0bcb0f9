"""Rows of y = H x at full size, computed by the oracle on sub-boxes.

The operator of the mixed system (eq. mixed-discretized) is local: a row
of H x involves x and the medium only within one cell of the row's
location.  So the oracle's assembled operator on a box of cells cut out of
the full grid -- with the medium (mu, lambda + mu, rho) and the attenuation
gamma of the full grid sliced to the box, and the box's own zero ghosts --
gives exactly the full grid's rows everywhere except next to a box side
that is not a side of the full domain (there the box's ghosts and its
one-sided averages differ).  Rows at least `margin` points from such a side
are kept; sides shared with the domain are exact (same zero ghosts, same
existing-cell averages).  Test infrastructure: only tests import this.
"""
import numpy as np

from oracle.elastic import ElasticSystem, abc_gamma, lame_from_velocities


def field_layout(n):
    """(shape slowest-first, flat offset) of u_1..u_d and p in [u | p]."""
    d = len(n)
    out, off = [], 0
    for k in range(d + 1):
        m = [n[a] + (1 if a == k else 0) for a in range(d)]
        shape = tuple(reversed(m))
        out.append((shape, off))
        off += int(np.prod(shape))
    return out


def window_rows(n, h, vp, vs, rho, omega, abc_width, abc_sides, x, lo, w, margin=2):
    """Oracle rows of H x on the box of cells [lo_a, lo_a + w_a) (x first).

    Returns (idx, y): flat indices into the full vector and the oracle's
    values there, for every row at least `margin` points away from each
    box side that lies inside the domain."""
    n = tuple(int(v) for v in n)
    d = len(n)
    lo = tuple(int(v) for v in lo)
    w = tuple(int(v) for v in w)
    assert all(0 <= lo[a] and lo[a] + w[a] <= n[a] for a in range(d))
    mu, lam_mu = lame_from_velocities(vp, vs, rho)
    gamma = abc_gamma(n, omega, abc_width, abc_sides)
    cells = tuple(slice(lo[a], lo[a] + w[a]) for a in reversed(range(d)))
    sub = ElasticSystem(w, h, rho=np.asarray(rho)[cells], omega=omega, mu=mu[cells],
                        lam_mu=lam_mu[cells], gamma=gamma[cells])
    full = field_layout(n)
    box = field_layout(w)
    xs, keep_idx, keep_loc = [], [], []
    for f in range(d + 1):
        shape, off = full[f]
        bshape, boff = box[f]
        sl = tuple(slice(lo[a], lo[a] + w[a] + (1 if a == f else 0)) for a in reversed(range(d)))
        xf = np.asarray(x)[off:off + int(np.prod(shape))].reshape(shape)
        xs.append(xf[sl].ravel())
        ok = np.ones(bshape, dtype=bool)
        for a in range(d):
            ax = d - 1 - a                       # array axis of grid axis a
            m = bshape[ax]
            i = np.arange(m)
            good = np.ones(m, dtype=bool)
            if lo[a] > 0:
                good &= i >= margin
            if lo[a] + w[a] < n[a]:
                good &= i <= m - 1 - margin
            ok &= good.reshape([m if b == ax else 1 for b in range(d)])
        loc = np.nonzero(ok.ravel())[0]
        coords = np.unravel_index(loc, bshape)
        gcoords = tuple(c + lo[d - 1 - ax] for ax, c in enumerate(coords))
        keep_idx.append(off + np.ravel_multi_index(gcoords, shape))
        keep_loc.append(boff + loc)
    y = sub.apply_H(np.concatenate(xs))
    return np.concatenate(keep_idx), y[np.concatenate(keep_loc)]
