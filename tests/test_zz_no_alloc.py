"""The allocation-free misfit entry point against eh_misfit (needs an
MI355X): the same adjoint right-hand side and misfit, bitwise, on two calls
in a row, the second with fewer sources and receivers (the fixed device
scratch keeps the first call's entries); an out-of-range receiver index
gives a NaN misfit instead of a fault; too many sources is an argument
error before any device work."""
import sys

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_15897_amd import ElasticHelmholtz
    wl = W.config(3, scale=16)                 # 32 x 32
    s = ElasticHelmholtz(wl.n, wl.h, wl.vp, wl.vs, wl.rho, wl.omega, levels=2, alpha=0.3,
                         abc_width=4, abc_sides=wl.abc_sides)
    yield wl, s
    s.close()


def _inputs(wl, s, nrhs, nrec, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((nrhs, s.ndof)) + 1j * rng.standard_normal((nrhs, s.ndof))
    rec = W.receiver_indices(wl.n, sorted(set(wl.receivers))[:nrec])
    d = rng.standard_normal((nrhs, nrec)) + 1j * rng.standard_normal((nrhs, nrec))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return dev(u), dev(rec), dev(d)


def test_noalloc_misfit_equals_misfit_on_two_calls(solver):
    wl, s = solver
    for nrhs, nrec, seed in ((6, 16, 1), (2, 5, 2)):
        say(f"misfit without allocation: {nrhs} sources, {nrec} receivers")
        u, rec, d = _inputs(wl, s, nrhs, nrec, seed)
        phi_ref, g_ref = s.misfit(u, rec, d)
        g = torch.full_like(u, 7.0 + 7.0j)                 # stale contents must be overwritten
        phi = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        s.misfit_noalloc(u, rec, d, g, phi)
        torch.cuda.synchronize()
        assert phi.item() == phi_ref
        assert torch.equal(g, g_ref)


def test_noalloc_misfit_bad_receiver_and_size(solver):
    from paper_2411_15897_amd.solver import EhelmError
    wl, s = solver
    u, rec, d = _inputs(wl, s, 2, 4, 3)
    rec[1] = s.ndof                                          # out of range: skipped on the device
    g = torch.empty_like(u)
    phi = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.misfit_noalloc(u, rec, d, g, phi)
    torch.cuda.synchronize()
    assert np.isnan(phi.item())
    big = torch.zeros((4097, s.ndof), dtype=torch.complex128, device="cuda")
    dbig = torch.zeros((4097, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(EhelmError, match="4096"):
        s.misfit_noalloc(big, rec, dbig, torch.empty_like(big), phi)
