"""GPU parity of the block-tridiagonal coarsest solve (needs an MI355X).

The coarsest level of every block is solved directly (Section 4.4.1).  The
oracle solves it by sparse LU (scipy's splu); the GPU factors it block-
tridiagonally over groups of planes.  Both are exact up to rounding, so the
results agree to 1e-10 relative (FP64), on the fine operators themselves
(one level: the cycle is the direct solve) and under Galerkin coarsening
with either intergrid, in 2D (coarsest 64 x 64) and 3D (coarsest 12^3).
"""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle.elastic import ElasticSystem, face_nodal
from oracle.multigrid import Hierarchy

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


def hetero_medium(n, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    vp = rng.uniform(2.0, 3.5, shape)
    vs = vp * rng.uniform(0.35, 0.55, shape)
    rho = rng.uniform(1.0, 2.0, shape)
    return vp, vs, rho


def make(n, seed=0, omega=0.7, abc=4, **kw):
    from paper_2411_15897_amd import ElasticHelmholtz
    dim = len(n)
    h = tuple(1.0 + 0.1 * a for a in range(dim))
    vp, vs, rho = hetero_medium(n, seed)
    sides = W.ABC_ALL[dim]
    gpu = ElasticHelmholtz(n, h, vp, vs, rho, omega, abc_width=abc, abc_sides=sides, **kw)
    sys_ = ElasticSystem(n, h, vp, vs, rho, omega, abc, sides)
    return gpu, sys_


def crand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def block_op(s, b, alpha):
    return s.H_p(alpha) if b == s.dim else s.A_block(b, alpha)


@pytest.mark.parametrize("n", [(64, 64), (40, 24), (12, 12, 12), (10, 6, 8)])
def test_direct_solve_of_fine_blocks(n):
    """One level: the cycle is the coarsest solve of the shifted fine block.
    Block-tridiagonal against splu (1e-10), and against the dense inverse
    where that fits (1e-10); two right-hand sides at once equal one at a
    time bitwise."""
    say("block-tridiagonal direct solve, one level", n)
    alpha = 0.3
    gpu, s = make(n, seed=1, levels=1, alpha=alpha, mg_precision=64, coarse_solver="bt")
    dense = None
    if max(int(np.prod(gpu.block_dims(b, 0))) for b in range(s.dim + 1)) <= 6000:
        dense, _ = make(n, seed=1, levels=1, alpha=alpha, mg_precision=64, coarse_solver="dense")
    for b in range(s.dim + 1):
        X = block_op(s, b, alpha).tocsc()
        f = crand((2, X.shape[0]), 5 + b)
        e = gpu.block_cycle(b, to_dev(f)).cpu().numpy()
        lu = spla.splu(X)
        for k in range(2):
            ref = lu.solve(f[k])
            assert rel(e[k], ref) <= 1e-10, (b, k, rel(e[k], ref))
            e1 = gpu.block_cycle(b, to_dev(f[k])).cpu().numpy()
            assert np.array_equal(e1, e[k])
        if dense is not None:
            ed = dense.block_cycle(b, to_dev(f)).cpu().numpy()
            assert rel(e, ed) <= 1e-10
    gpu.close()
    if dense is not None:
        dense.close()


@pytest.mark.parametrize("n,intergrid,levels", [
    ((128, 128), "full", 2),     # coarsest 64 x 64: line pairs along the cell-centred axes
    ((128, 128), "mixed", 2),
    ((128, 64), "full", 3),
    ((24, 24, 24), "mixed", 2),  # coarsest 12^3: plane groups of one
    ((24, 24, 24), "full", 2),   # plane pairs along cell-centred axes
])
def test_cycle_with_block_tridiagonal_coarsest(n, intergrid, levels):
    """A full cycle (V(1,2) in 2D, V(2,2) in 3D) whose coarsest Galerkin
    level is solved block-tridiagonally, against the oracle's cycle with
    splu on the coarsest level (FP64, 1e-10); complex64 multigrid within
    1e-5."""
    say("cycle with block-tridiagonal coarsest", n, intergrid, levels)
    alpha = 0.3
    dim = len(n)
    nu = (1, 2) if dim == 2 else (2, 2)
    damping = (0.8, 0.8, 0.3) if dim == 2 else (0.8, 0.8, 0.2)
    kw = dict(levels=levels, alpha=alpha, nu=nu, damping=damping, intergrid=intergrid, coarse_solver="bt")
    gpu, s = make(n, seed=2, mg_precision=64, **kw)
    g32, _ = make(n, seed=2, mg_precision=32, **kw)
    for b in range(dim + 1):
        X = block_op(s, b, alpha)
        nodal = tuple(False for _ in range(dim)) if b == dim else face_nodal(dim, b)
        mg = Hierarchy(X, s.n, nodal, levels, damping=damping, nu=nu, intergrid=intergrid)
        f = crand(X.shape[0], 30 + b)
        ref = mg(f)
        e = gpu.block_cycle(b, to_dev(f)).cpu().numpy()
        assert rel(e, ref) <= 1e-10, (b, rel(e, ref))
        e32 = g32.block_cycle(b, to_dev(f)).cpu().numpy()
        say(f"  block {b}: FP64 {rel(e, ref):.2e}, complex64 multigrid {rel(e32, ref):.2e}")
        assert rel(e32, ref) <= 1e-5
    gpu.close()
    g32.close()


@pytest.mark.parametrize("intergrid", ["mixed", "full"])
def test_wide_groups_batched(intergrid):
    """Coarsest 20^3: groups of one plane (400-420 unknowns) with the mixed
    intergrid, plane pairs (800-840) with full weighting, so the forward
    and back steps and the S_I^-1 f_I launch take their columns in several
    chunks (320 columns per chunk with 5-8 right-hand sides, 640 with
    fewer).  Each right-hand side of a batch of 7, and one alone, against
    the oracle's cycle with splu on the coarsest level (FP64, 1e-10)."""
    say("block-tridiagonal wide groups, batched", intergrid)
    n, alpha = (40, 40, 40), 0.3
    nu, damping = (2, 2), (0.8, 0.8, 0.2)
    kw = dict(levels=2, alpha=alpha, nu=nu, damping=damping, intergrid=intergrid, coarse_solver="bt")
    gpu, s = make(n, seed=5, mg_precision=64, **kw)
    for b in range(4):
        X = block_op(s, b, alpha)
        nodal = (False,) * 3 if b == 3 else face_nodal(3, b)
        mg = Hierarchy(X, s.n, nodal, 2, damping=damping, nu=nu, intergrid=intergrid)
        f = crand((7, X.shape[0]), 50 + b)
        e = gpu.block_cycle(b, to_dev(f)).cpu().numpy()
        e1 = gpu.block_cycle(b, to_dev(f[:1])).cpu().numpy()[0]
        errs = [rel(e[k], mg(f[k])) for k in range(7)]
        say(f"  block {b}: max rel err {max(errs):.1e}")
        assert max(errs) <= 1e-10, (b, errs)
        assert rel(e1, e[0]) <= 1e-13
    gpu.close()


@pytest.mark.parametrize("nrhs", [3, 7, 9])
def test_batch_equals_single(nrhs):
    """Chunks of 4 or 8 right-hand sides per workgroup (and a ragged last
    chunk) give each right-hand side bitwise what it gets alone, through
    the whole preconditioner."""
    say("block-tridiagonal batch", nrhs)
    n = (48, 32)
    gpu, s = make(n, seed=3, levels=2, alpha=0.4, mg_precision=32, coarse_solver="bt")
    r = crand((nrhs, s.ndof), 4)
    zb = gpu.apply_preconditioner(to_dev(r)).cpu().numpy()
    for k in range(nrhs):
        zk = gpu.apply_preconditioner(to_dev(r[k:k + 1])).cpu().numpy()[0]
        assert np.array_equal(zb[k], zk), k
    gpu.close()
