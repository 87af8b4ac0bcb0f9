"""Write the oracle's own FGMRES iteration counts for a benchmark workload.

Runs the CPU FP64 oracle (sparse V-cycles with the workload's settings,
modified Gram-Schmidt FGMRES, splu on the coarsest level) to a true
relative residual of 1e-6 on every source of the workload, in worker
processes forked after one setup, and writes
``oracle_iterations_<workload name>.json`` beside this script: per source
the iteration count and the final true residual, plus the setup and
per-iteration seconds on this host.  The benchmark's CPU baseline
extrapolates with these counts (they are the oracle's, not the GPU's).

Usage: python tests/golden/make_oracle_iterations.py [config] [workers]
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

_STATE = {}


def _solve(q):
    from oracle.fgmres import fgmres
    wl, H, M, b = _STATE["wl"], _STATE["H"], _STATE["M"], _STATE["b"]
    t0 = time.perf_counter()
    res = fgmres(lambda x: H @ x, M, b[q], restart=wl.restart, tol=wl.tol, maxit=2000)
    dt = time.perf_counter() - t0
    print(f"source {q}: {res.iters} iterations, relres {res.relres_true:.3e}, {dt:.1f} s", flush=True)
    return {"source": q, "iters": int(res.iters), "relres_true": float(res.relres_true),
            "converged": bool(res.converged), "seconds": dt}


def main():
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle.elastic import ElasticSystem
    from oracle.precond import BlockAcoustic

    k = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else 4
    wl = W.config(k)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        s = ElasticSystem(wl.n, wl.h, wl.vp, wl.vs, wl.rho, wl.omega, wl.abc_width, wl.abc_sides)
        H = s.H()
        M = BlockAcoustic(s, alpha=wl.alpha, solver="mg", levels=wl.levels, cycle="V", nu=wl.nu,
                          damping=wl.damping, intergrid=wl.intergrid)
        setup = time.perf_counter() - t0
        print(f"{wl.name}: oracle setup {setup:.1f} s", flush=True)
        _STATE.update(wl=wl, H=H, M=M, b=W.point_source_rhs(wl.n, wl.h, wl.sources))
        nsrc = len(wl.sources)
        with mp.get_context("fork").Pool(workers) as pool:
            rows = pool.map(_solve, range(nsrc), chunksize=1)
    its = [r["iters"] for r in rows]
    out = {
        "workload": wl.name,
        "what": ("iterations of the CPU FP64 oracle (FGMRES(%d) with modified Gram-Schmidt, block-acoustic "
                 "preconditioner with one V(%d,%d) cycle per block, %d levels, shift %.2f, splu on the "
                 "coarsest level) to a true relative residual of %.0e, x0 = 0"
                 % (wl.restart, wl.nu[0], wl.nu[1], wl.levels, wl.alpha, wl.tol)),
        "script": "tests/golden/make_oracle_iterations.py %d %d" % (k, workers),
        "host": {"nproc": os.cpu_count(), "workers": workers, "threads_per_worker": 1},
        "setup_seconds": setup,
        "seconds_per_iteration": sum(r["seconds"] for r in rows) / max(sum(its), 1),
        "iters_mean": sum(its) / len(its),
        "iters_min": min(its),
        "iters_max": max(its),
        "sources": rows,
    }
    path = os.path.join(HERE, f"oracle_iterations_{wl.name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: iterations {min(its)}..{max(its)}, mean {out['iters_mean']:.2f}")


if __name__ == "__main__":
    main()
