"""Dropping converged right-hand sides from the batch (drop_converged).

At a restart whose true residuals show some right-hand sides finished, the
solver gathers the others into the first slots and launches only over them.
Every kernel's arithmetic per right-hand side is independent of the batch
around it, so the solution, the iteration counts and the residuals must be
bitwise those of the run in which every launch covers the whole batch.
"""
import sys

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_15897_amd import _native
    _native.lib()          # fails loudly when the library is missing


def medium(n, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    vp = rng.uniform(2.0, 3.5, shape)
    vs = vp * rng.uniform(0.35, 0.55, shape)
    rho = rng.uniform(1.0, 2.0, shape)
    return vp, vs, rho


def solver(n, drop, **kw):
    from paper_2411_15897_amd import ElasticHelmholtz
    dim = len(n)
    h = tuple(1.0 + 0.1 * a for a in range(dim))
    vp, vs, rho = medium(n, 23)
    return ElasticHelmholtz(n, h, vp, vs, rho, 0.7, abc_width=4, abc_sides=W.ABC_ALL[dim],
                            drop_converged=drop, **kw)


def mixed_rhs(n, ndof, seed):
    """Right-hand sides that finish in different restart cycles: point
    forces at the centre and near a corner, a zero one, white noise, a
    smooth field and a scaled copy of the first."""
    h = tuple(1.0 + 0.1 * a for a in range(len(n)))
    mid = tuple(v // 2 for v in n)
    corner = tuple(2 for _ in n)
    pts = W.point_source_rhs(n, h, [(0, mid), (len(n) - 1, corner)])
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(ndof) + 1j * rng.standard_normal(ndof)
    smooth = np.cumsum(rng.standard_normal(ndof)) * (1.0 + 0.5j) / np.sqrt(ndof)
    return np.stack([pts[0], np.zeros(ndof), noise, pts[1], smooth, 1e3 * pts[0]])


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("n,kw", [
    ((96, 80), dict(levels=3, alpha=0.4, restart=4, mg_precision=32)),
    ((96, 80), dict(levels=3, alpha=0.4, restart=3, mg_precision=64, graphs=False)),
    ((12, 8, 10), dict(levels=2, alpha=0.4, restart=4, mg_precision=32, intergrid="mixed")),
])
def test_drop_converged_equals_full_batch(n, kw):
    """x, iteration counts and residuals bitwise equal with and without the
    drop; the counts spread over several restart cycles (so drops happen,
    the zero right-hand side at the first start); a second, smaller solve on
    the context that dropped (graphs re-captured for the new batch) equals
    the same solve on the other context."""
    say("drop converged", n, kw)
    a = solver(n, True, **kw)
    b = solver(n, False, **kw)
    rhs = to_dev(mixed_rhs(n, a.ndof, 5))
    xa, ia = a.solve(rhs, tol=1e-8, maxit=400)
    xb, ib = b.solve(rhs, tol=1e-8, maxit=400)
    its = [i["iters"] for i in ia]
    say("  iterations", its)
    assert all(i["converged"] for i in ia)
    assert ia[1]["iters"] == 0
    nz = [v for v in its if v > 0]
    assert max(nz) - min(nz) >= kw["restart"], its
    assert ia == ib
    assert torch.equal(xa, xb)
    assert torch.all(xa[1] == 0)
    sub = rhs[2:4].contiguous()
    xa2, ia2 = a.solve(sub, tol=1e-8, maxit=400)
    xb2, ib2 = b.solve(sub, tol=1e-8, maxit=400)
    assert ia2 == ib2 and torch.equal(xa2, xb2)
    assert ia2 == ia[2:4] and torch.equal(xa2, xa[2:4])
    a.close()
    b.close()


def test_drop_converged_block_solve():
    """The single-block solver drops finished right-hand sides the same way
    (the zero one at the first start): bitwise equal to the full batch."""
    say("drop converged, block solve")
    n = (96, 80)
    kw = dict(levels=3, alpha=0.8, restart=20, mg_precision=32)
    a = solver(n, True, **kw)
    b = solver(n, False, **kw)
    npts = int(np.prod(a.block_dims(2, 0)))
    rng = np.random.default_rng(8)
    f = np.zeros((4, npts), dtype=np.complex128)
    f[0, npts // 2] = 1.0
    f[2] = rng.standard_normal(npts) + 1j * rng.standard_normal(npts)
    f[3] = np.cumsum(rng.standard_normal(npts)) / np.sqrt(npts)
    xa, ia = a.block_solve(2, to_dev(f), tol=1e-6, maxit=300)
    xb, ib = b.block_solve(2, to_dev(f), tol=1e-6, maxit=300)
    say("  iterations", [i["iters"] for i in ia])
    assert ia[1]["iters"] == 0 and ia[1]["converged"]
    assert ia == ib and torch.equal(xa, xb)
    a.close()
    b.close()
