"""FWI gradient through torch.autograd (needs an MI355X).

The layered medium with 16 top sources and receivers every second face
(the 512^2 FWI workload, here at 128^2 so the test runs in seconds), the
observed data from the medium with a smoothed 2% perturbation of vp and vs.
The autograd gradient is checked against central finite differences of the
same GPU misfit on 10 random directions (relative step 1e-6, complex128
solves to 1e-12), and against the oracle's gradient with direct solves at
128^2 with all 16 sources.  At the full 512^2 size the same finite-
difference check runs on 10 directions.  A forward or adjoint solve that
stops short of its tolerance raises instead of returning a gradient.
"""
import sys

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def problem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_15897_amd import _native
    _native.lib()
    wl = W.config(3, scale=4)                  # 128 x 128, 16 sources, 256 -> 64 receivers
    recs = sorted(set(wl.receivers))
    rng = np.random.default_rng(2)
    from workloads import _smooth_field
    pert = 0.02 * _smooth_field(rng, wl.vp.shape, 5.0)
    vp_true, vs_true = wl.vp * (1 + pert), wl.vs * (1 + pert)
    b = W.point_source_rhs(wl.n, wl.h, wl.sources)
    rec = W.receiver_indices(wl.n, recs)
    geom = dict(n=wl.n, h=wl.h, omega=wl.omega, levels=3, alpha=0.3, mg_precision=64,
                restart=20, abc_width=wl.abc_width // 4, abc_sides=wl.abc_sides, tol=1e-12,
                maxit=3000)
    from paper_2411_15897_amd import ElasticHelmholtz
    g2 = dict(geom); tol = g2.pop("tol"); maxit = g2.pop("maxit")
    n, h, om = g2.pop("n"), g2.pop("h"), g2.pop("omega")
    s = ElasticHelmholtz(n, h, vp_true, vs_true, wl.rho, om, **g2)
    bt = torch.from_numpy(b).cuda()
    u, info = s.solve(bt, tol=tol, maxit=maxit)
    assert all(i["converged"] for i in info)
    d_obs = u[:, torch.from_numpy(rec).cuda()].contiguous()
    s.close()
    return wl, geom, bt, torch.from_numpy(rec).cuda(), d_obs


def test_autograd_gradient_matches_finite_differences(problem):
    from paper_2411_15897_amd.fwi import misfit
    wl, geom, b, rec, d_obs = problem
    vp = torch.tensor(wl.vp, dtype=torch.float64, requires_grad=True)
    vs = torch.tensor(wl.vs, dtype=torch.float64, requires_grad=True)
    rho = torch.tensor(wl.rho, dtype=torch.float64, requires_grad=True)
    phi = misfit(vp, vs, rho, geom, b, rec, d_obs)
    phi.backward()
    say(f"phi = {phi.item():.6e}")
    rng = np.random.default_rng(7)
    eps = 1e-6
    worst = 0.0
    for t in range(10):
        dirs = [m * rng.standard_normal(m.shape) for m in (wl.vp, wl.vs, wl.rho)]
        with torch.no_grad():
            def at(sg):
                return misfit(*(torch.tensor(m + sg * eps * d) for m, d in
                                zip((wl.vp, wl.vs, wl.rho), dirs)), geom, b, rec, d_obs).item()
            fd = (at(1.0) - at(-1.0)) / (2 * eps)
        an = sum(float((g.grad.numpy() * d).sum()) for g, d in zip((vp, vs, rho), dirs))
        err = abs(fd - an) / abs(an)
        worst = max(worst, err)
        say(f"  direction {t}: fd {fd:.10e} adjoint {an:.10e} rel err {err:.2e}")
        assert err <= 1e-5
    say(f"worst relative error over 10 directions: {worst:.2e}")


def test_autograd_gradient_matches_oracle(problem):
    """The 128 x 128 workload of the finite-difference test (16 sources,
    64 receivers): the GPU autograd gradient against the oracle's gradient
    with direct (splu) forward and adjoint solves, to 1e-8 relative."""
    from oracle.fwi import gradient as ogradient
    from paper_2411_15897_amd.fwi import misfit
    wl, geom, b, rec, d_obs = problem
    g = dict(geom, tol=1e-13, maxit=4000)
    vp = torch.tensor(wl.vp, requires_grad=True)
    vs = torch.tensor(wl.vs, requires_grad=True)
    rho = torch.tensor(wl.rho, requires_grad=True)
    phi = misfit(vp, vs, rho, g, b, rec, d_obs)
    phi.backward()
    phi_o, (gvp, gvs, grho), _, _ = ogradient(wl.n, wl.h, wl.vp, wl.vs, wl.rho, wl.omega, geom["abc_width"],
                                              wl.abc_sides, b.cpu().numpy(), rec.cpu().numpy(),
                                              d_obs.cpu().numpy())
    say(f"  phi gpu {phi.item():.12e} oracle {phi_o:.12e}")
    assert abs(phi.item() - phi_o) <= 1e-9 * abs(phi_o)
    for t, o in ((vp, gvp), (vs, gvs), (rho, grho)):
        a = t.grad.numpy().ravel()
        err = np.linalg.norm(a - o) / np.linalg.norm(o)
        say(f"  gradient rel err {err:.2e}")
        assert err <= 1e-8


def test_unconverged_solve_raises(problem):
    """maxit too small for the tolerance: the misfit refuses to return."""
    from paper_2411_15897_amd.fwi import misfit
    from paper_2411_15897_amd.solver import EhelmError
    wl, geom, b, rec, d_obs = problem
    g = dict(geom, maxit=3)
    vp, vs, rho = (torch.tensor(m) for m in (wl.vp, wl.vs, wl.rho))
    with pytest.raises(EhelmError, match="forward solve did not reach tol"):
        misfit(vp, vs, rho, g, b, rec, d_obs)


@pytest.mark.timeout(900)
def test_gradient_full_size_512_finite_differences():
    """The 512 x 512 FWI workload at full size (16 top sources, 256
    receivers, observed data from the medium with a smoothed 2% perturbation
    of vp and vs, 5 levels, alpha 0.7): the autograd gradient against central
    finite differences of the same GPU misfit along 10 random directions
    (relative step 1e-6; FP64 multigrid, FGMRES(20) to 1e-12 so that the
    differences resolve the derivative)."""
    say("full-size FWI gradient 512^2 x 16")
    from paper_2411_15897_amd import ElasticHelmholtz
    from paper_2411_15897_amd.fwi import misfit
    from workloads import _smooth_field
    wl = W.config(3)
    recs = sorted(set(wl.receivers))
    assert len(wl.sources) == 16 and len(recs) == 256
    pert = 0.02 * _smooth_field(np.random.default_rng(2), wl.vp.shape, 20.0)
    b = torch.from_numpy(W.point_source_rhs(wl.n, wl.h, wl.sources)).cuda()
    rec = torch.from_numpy(W.receiver_indices(wl.n, recs)).cuda()
    geom = dict(n=wl.n, h=wl.h, omega=wl.omega, levels=wl.levels, alpha=wl.alpha, mg_precision=64,
                restart=20, abc_width=wl.abc_width, abc_sides=wl.abc_sides, tol=1e-12, maxit=3000)
    g2 = {k: v for k, v in geom.items() if k not in ("n", "h", "omega", "tol", "maxit")}
    s = ElasticHelmholtz(wl.n, wl.h, wl.vp * (1 + pert), wl.vs * (1 + pert), wl.rho, wl.omega, **g2)
    u, info = s.solve(b, tol=geom["tol"], maxit=geom["maxit"])
    assert all(i["converged"] for i in info)
    d_obs = u[:, rec].contiguous()
    s.close()
    del u
    vp = torch.tensor(wl.vp, dtype=torch.float64, requires_grad=True)
    vs = torch.tensor(wl.vs, dtype=torch.float64, requires_grad=True)
    rho = torch.tensor(wl.rho, dtype=torch.float64, requires_grad=True)
    phi = misfit(vp, vs, rho, geom, b, rec, d_obs)
    phi.backward()
    say(f"  phi = {phi.item():.6e}, iters {info[0]['iters']}")
    rng = np.random.default_rng(8)
    eps = 1e-6
    worst = 0.0
    for t in range(10):
        dirs = [m * rng.standard_normal(m.shape) for m in (wl.vp, wl.vs, wl.rho)]
        with torch.no_grad():
            def at(sg):
                return misfit(*(torch.tensor(m + sg * eps * d) for m, d in
                                zip((wl.vp, wl.vs, wl.rho), dirs)), geom, b, rec, d_obs).item()
            fd = (at(1.0) - at(-1.0)) / (2 * eps)
        an = sum(float((g.grad.numpy() * d).sum()) for g, d in zip((vp, vs, rho), dirs))
        err = abs(fd - an) / abs(an)
        worst = max(worst, err)
        say(f"  direction {t}: fd {fd:.10e} adjoint {an:.10e} rel err {err:.2e}")
        assert err <= 1e-5
    say(f"  worst relative error over 10 directions: {worst:.2e}")
