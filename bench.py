"""Benchmark: seconds per right-hand side to a relative residual of 1e-6.

One step is one full solve (FGMRES from x = 0 to ||b - Hx||/||b|| < 1e-6,
block-acoustic preconditioner with one multigrid V-cycle per block) of the
1024 x 1024 layered + random medium with one top point source, with all
inputs resident in HBM.  The headline form is the complex64 multigrid under
FP64 FGMRES; the plain FP64 form is timed beside it.  The line also carries
the roofline figure of the V-cycle kernels, which take most of the solve
(every multigrid launch event-timed over the timed solves: algorithmic
bytes over launch time against the HBM peak), the per-class split of one
solve, and the CPU oracle's rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(wl, iters_ref, n_iters):
    """The oracle (NumPy/SciPy FP64, single thread) on the same workload:
    setup excluded, `n_iters` FGMRES iterations timed, extrapolated to the
    GPU's FP64 iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle.elastic import ElasticSystem
    from oracle.fgmres import fgmres
    from oracle.precond import BlockAcoustic

    with threadpool_limits(1):
        s = ElasticSystem(wl.n, wl.h, wl.vp, wl.vs, wl.rho, wl.omega, wl.abc_width, wl.abc_sides)
        H = s.H()
        M = BlockAcoustic(s, alpha=wl.alpha, solver="mg", levels=wl.levels, cycle="V",
                          nu=wl.nu, damping=wl.damping)
        b = W.point_source_rhs(wl.n, wl.h, wl.sources)[0]
        t0 = time.perf_counter()
        res = fgmres(lambda x: H @ x, M, b, restart=wl.restart, tol=wl.tol, maxit=n_iters)
        dt = time.perf_counter() - t0
    per_it = dt / max(res.iters, 1)
    return {
        "value": per_it * iters_ref,
        "unit": "s/RHS",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{res.iters} FGMRES iterations of the oracle (FP64 sparse V-cycles, "
                   f"setup excluded) on the same workload ({wl.name}), {per_it:.3f} s/iteration, "
                   f"extrapolated to the GPU FP64 iteration count {iters_ref}"),
        "host": {"nproc": os.cpu_count(), "cpu": host_cpu_model()},
    }


def host_cpu_model():
    """The host CPU's model name (Linux), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# the multigrid cycles proper (smoothing, residuals, transfers, coarsest
# solve), as opposed to the operator, the distributor, the coupling and the
# Krylov passes around them: the event-timer classes of the "vcycle" group
VCYCLE_CLASSES = ("fine_first", "fine_sweep", "fine_resid", "fine_down", "fine_up", "coarse", "coarse_down",
                  "coarse_up", "restrict", "prolong", "dense")
TIMER_GROUPS = {"vcycle": VCYCLE_CLASSES}

# Kernels of each event-timer class (substrings of the demangled names
# rocprofv3 prints) and, where a timed launch spans several dispatches, the
# ones that open a timed launch (a Gram-Schmidt pass is k_gs plus its
# fixed-order reduction).
CLASS_KERNELS = {
    "krylov": (("eh::k_gs<", "eh::k_reduce_partials", "eh::k_xupdate<"), ("eh::k_gs<", "eh::k_xupdate<")),
    "fine_down": (("eh::k_fdown<float, true", "eh::k_fdown<double, true"), None),
    "fine_up": (("eh::k_fup<float, true", "eh::k_fup<double, true"), None),
    "coarse_down": (("eh::k_fdown<float, false", "eh::k_fdown<double, false"), None),
    "coarse_up": (("eh::k_fup<float, false", "eh::k_fup<double, false"), None),
    "coarse": (("eh::k_gstencil<",), None),
    "operator": (("eh::k_op_face<", "eh::k_op_cell<"), ("eh::k_op_cell<",)),   # one H apply = 3 (4) fields
    "distribute": (("eh::k_distribute<",), None),
    "couple": (("eh::k_gcouple<",), None),
    "dense": (("eh::k_gdense<",), None),
    # every timed multigrid kernel: the V-cycles of the three (four) blocks
    "vcycle": (("eh::k_fdown<", "eh::k_fup<", "eh::k_gdense<", "eh::k_gstencil<", "eh::k_gfine<",
                "eh::k_gtransfer<"), None),
}
CLASS_SOURCES = {
    "krylov": ["paper_2411_15897_amd/csrc/eh_krylov_kernels.h", "paper_2411_15897_amd/csrc/eh_common.h"],
}
DEFAULT_SOURCES = ["paper_2411_15897_amd/csrc/eh_fused_kernels.h", "paper_2411_15897_amd/csrc/eh_group_kernels.h",
                   "paper_2411_15897_amd/csrc/eh_mg_kernels.h", "paper_2411_15897_amd/csrc/eh_op_kernels.h",
                   "paper_2411_15897_amd/csrc/eh_common.h"]




def timer_classes(kernel):
    """The event-timer classes of a class name or a group name."""
    from paper_2411_15897_amd._native import KERNEL_CLASSES
    names = TIMER_GROUPS.get(kernel, (kernel,))
    bad = [k for k in names if k not in KERNEL_CLASSES]
    if bad:
        raise SystemExit(f"bench.py: unknown kernel class {bad}")
    return list(names)


def vcycle_summary(split_bytes):
    """Algorithmic GB/s of all V-cycle launches of one event-timed solve
    (sum of bytes / sum of launch durations) against the HBM peak, and the
    V-cycles' share of the event-timed solve."""
    if not split_bytes:
        return None
    ms = sum(split_bytes[k][0] for k in VCYCLE_CLASSES if k in split_bytes)
    nbytes = sum(split_bytes[k][1] for k in VCYCLE_CLASSES if k in split_bytes)
    total = sum(v[0] for v in split_bytes.values())
    if ms <= 0:
        return None
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"classes": [k for k in VCYCLE_CLASSES if k in split_bytes], "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "ms_one_solve": round(ms, 3),
            "share_of_solve": ms / total}


def sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def pmc_summary(fetch_csv, write_csv, kernel, workload):
    """HBM traffic per timed launch of a kernel class from a FETCH_SIZE and a
    WRITE_SIZE rocprofv3 counter run (KiB per dispatch), each scaled by what
    the same counter reads for the 1 GiB calibration copy of the same run
    (the run's first copy dispatch: it precedes the solver's own copies).
    Only the run's last solve counts: the dispatches after the last copy
    (each solve starts by copying b into the first basis column and copies
    nothing else), so set-up and tuning launches do not enter."""
    import csv
    members, leads = CLASS_KERNELS[kernel]
    leads = leads or members
    rec = {"kernel_class": kernel, "kernels": ", ".join(members), "workload": workload}
    total = 0.0
    for tag, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        copies = sorted((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in rows
                        if "__amd_rocclr_copyBuffer" in r["Kernel_Name"])
        if len(copies) < 2:
            raise SystemExit(f"bench.py: {path} holds {len(copies)} copy dispatches; a run with "
                             "--copy-calibration and at least one solve has two or more")
        ref = copies[0][1]                              # the 1 GiB calibration copy
        scale = (1 << 30) / 1024.0 / ref
        last = copies[-1][0]                            # start of the last solve
        cls = [r for r in rows if int(r["Dispatch_Id"]) > last and any(m in r["Kernel_Name"] for m in members)]
        nlaunch = sum(1 for r in cls if any(m in r["Kernel_Name"] for m in leads))
        kib = sum(float(r["Counter_Value"]) for r in cls) / max(nlaunch, 1)
        rec[f"{tag}_kib_per_launch_raw"] = kib
        rec[f"copy_{tag}_kib"] = ref
        rec[f"{tag}_scale"] = scale
        rec[f"launches_{tag}"] = nlaunch
        rec[f"dispatches_{tag}"] = len(cls)
        total += kib * scale * 1024.0
    rec["copy_reference"] = "torch copy of 1 GiB (__amd_rocclr_copyBuffer) in the same runs"
    rec["launches_counted"] = "the dispatches of the run's last solve (after its last copy)"
    rec["traffic_bytes_per_launch"] = total
    rec["source_files"] = CLASS_SOURCES.get(kernel, DEFAULT_SOURCES)
    rec["source_sha256"] = sources_sha256(rec["source_files"])
    run = "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp64 --copy-calibration"
    fdir, wdir = os.path.dirname(fetch_csv), os.path.dirname(write_csv)
    rec["commands"] = [
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {fdir} -o run -- {run}",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {wdir} -o run -- {run}",
        f"python3 bench.py --roofline-kernel {kernel} --pmc-summary {fetch_csv} {write_csv}",
    ]
    return rec


def trace_summary(trace_csv, solves):
    """Per kernel class (and the vcycle group): launches and average
    duration over the last `solves` solves of a rocprofv3 --kernel-trace
    run of this script with --no-fp64 --no-cpu-baseline (its last solves
    are the event-timed ones; each solve starts with its one copy)."""
    import csv
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Dispatch_Id"]))
    copies = [i for i, r in enumerate(rows) if "__amd_rocclr_copyBuffer" in r["Kernel_Name"]]
    if solves < 1 or len(copies) < solves:
        raise SystemExit(f"bench.py: {trace_csv} holds {len(copies)} solves (copy dispatches), "
                         f"fewer than --steps {solves}")
    tail = rows[copies[-solves] + 1:]
    out = {}
    for k, (members, leads) in CLASS_KERNELS.items():
        leads = leads or members
        sel = [r for r in tail if any(m in r["Kernel_Name"] for m in members)]
        if not sel:
            continue
        n = sum(1 for r in sel if any(m in r["Kernel_Name"] for m in leads))
        ns = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in sel)
        out[k] = {"dispatches": len(sel), "launches": n, "total_ms": ns * 1e-6,
                  "avg_us": ns * 1e-3 / max(n, 1)}
    return out


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs, or None when none was recorded
    for that kernel class and workload or the kernel sources changed since
    (sha256 mismatch)."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.txt")):
        try:
            rec = json.load(open(path))
        except (OSError, ValueError):
            continue
        if rec.get("kernel_class") != kernel or rec.get("workload") != workload:
            continue
        if sources_sha256(rec["source_files"]) != rec["source_sha256"]:
            return None
        return rec["traffic_bytes_per_launch"]
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--restart", type=int, default=None)
    ap.add_argument("--roofline-kernel", default="vcycle",
                    help="kernel class (or the group vcycle: every multigrid kernel) for the roofline figure")
    ap.add_argument("--cpu-iters", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB with torch before the solves (reference dispatch for HBM counters)")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="no GPU work: per-class launches and average durations over the last --steps solves "
                         "of a rocprofv3 --kernel-trace run of this script (--no-fp64 --no-cpu-baseline)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU work: print the HBM traffic record of --roofline-kernel from the counter "
                         "CSVs of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script")
    args = ap.parse_args()
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary, args.steps), indent=1))
        return
    if args.pmc_summary:
        import workloads as W
        print(json.dumps(pmc_summary(*args.pmc_summary, args.roofline_kernel, W.config(args.config).name),
                         indent=1))
        return
    if args.gpus != 1:
        print("bench.py: this solver runs on one GPU only; several GPUs would each take a share of "
              "the sources, with one all-reduce of the gradient at the end",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2411_15897_amd import ElasticHelmholtz

    wl = W.config(args.config)
    if args.levels:
        wl.levels = args.levels
    if args.alpha is not None:
        wl.alpha = args.alpha
    if args.restart:
        wl.restart = args.restart
    dev = torch.device("cuda:0")
    b = torch.from_numpy(W.point_source_rhs(wl.n, wl.h, wl.sources)).to(dev)
    nrhs = b.shape[0]

    def make(prec):
        return ElasticHelmholtz(wl.n, wl.h, wl.vp, wl.vs, wl.rho, wl.omega, levels=wl.levels,
                                nu=wl.nu, damping=wl.damping, alpha=wl.alpha, mg_precision=prec,
                                restart=wl.restart, abc_width=wl.abc_width,
                                abc_sides=wl.abc_sides, intergrid=wl.intergrid)

    def timed(solver, steps, warmup, kernel=None):
        for w in range(warmup):
            _, info = solver.solve(b, tol=wl.tol, maxit=5000)
            log(f"warmup {w}: iters {info[0]['iters']} relres {info[0]['relres_true']:.2e}")
        classes = timer_classes(kernel) if kernel else []
        for k in classes:
            solver.timer_read(k)               # drop anything recorded before
        if classes:
            solver.timer_enable(classes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for k in range(steps):
            _, info = solver.solve(b, tol=wl.tol, maxit=5000)
            infos.append(info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = None
        if classes:
            reads = [solver.timer_read(k) for k in classes]
            kt = tuple(sum(r[i] for r in reads) for i in range(3))
        solver.timer_enable([])
        log(f"timed {steps} solves in {dt:.3f} s, iters {[i[0]['iters'] for i in infos]}")
        return dt, infos, kt

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)       # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"workload {wl.name}: n={wl.n} omega={wl.omega:.4f} levels={wl.levels} alpha={wl.alpha}")
    t_setup = time.perf_counter()
    s32 = make(32)
    torch.cuda.synchronize()
    log(f"setup (complex64 multigrid) {time.perf_counter() - t_setup:.2f} s")
    kernel = args.roofline_kernel
    split = {}
    split_bytes = {}
    # one untimed solve with every kernel class event-timed: the split of
    # the solve over the classes
    from paper_2411_15897_amd._native import KERNEL_CLASSES
    s32.timer_enable(list(KERNEL_CLASSES))
    s32.solve(b, tol=wl.tol, maxit=5000)
    for k in KERNEL_CLASSES:
        n_, ms_, by_ = s32.timer_read(k)
        if n_:
            split[k] = {"launches": n_, "ms": round(ms_, 3),
                        "GB_s": round(by_ / (ms_ * 1e-3) / 1e9, 1)}
            split_bytes[k] = (ms_, by_)
    s32.timer_enable([])
    log(f"per-class split of one solve: {json.dumps(split)}")
    # value: the solve as it runs (Arnoldi steps replayed from HIP graphs)
    dt32, inf32, _ = timed(s32, args.steps, args.warmup, None)
    # roofline: the same K solves again with every launch of the roofline
    # class (default: all V-cycle kernels) bracketed by HIP events on the
    # solver's stream (plain launches; the kernels are the same, only the
    # launch path differs)
    _, _, kt = timed(s32, args.steps, 0, kernel)
    it32 = inf32[-1][0]["iters"]
    rel32 = max(i[0]["relres_true"] for i in inf32)
    s32.close()
    sec32 = dt32 / (args.steps * nrhs)

    fp64 = None
    it64 = it32
    if not args.no_fp64:
        # the plain form: complex128 multigrid, one right-hand side per solve
        s64 = make(64)
        if nrhs == 1:
            dt64, inf64, _ = timed(s64, max(1, min(args.steps, 2)), 1)
            it64 = inf64[-1][0]["iters"]
            fp64 = {"form": "complex128 multigrid, single RHS",
                    "s_per_rhs": dt64 / max(1, min(args.steps, 2)), "iters": it64,
                    "relres_true": max(i[0]["relres_true"] for i in inf64)}
        else:
            sample = list(range(min(nrhs, 2)))
            s64.solve(b[0:1], tol=wl.tol, maxit=5000)          # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            inf64 = [s64.solve(b[q:q + 1], tol=wl.tol, maxit=5000)[1][0] for q in sample]
            torch.cuda.synchronize()
            dt64 = time.perf_counter() - t0
            it64 = max(i["iters"] for i in inf64)
            fp64 = {"form": f"complex128 multigrid, single RHS, sources solved one at a time "
                            f"(first {len(sample)} of {nrhs} timed)",
                    "s_per_rhs": dt64 / len(sample), "iters": it64,
                    "relres_true": max(i["relres_true"] for i in inf64)}
            log(f"fp64 single-RHS solves: {dt64 / len(sample):.3f} s per RHS, iters {[i['iters'] for i in inf64]}")
        fp64["value_speedup"] = fp64["s_per_rhs"] / sec32
        s64.close()

    launches, ms, nbytes = kt
    avg_ms = ms / max(launches, 1)
    achieved = (nbytes / max(launches, 1)) / (avg_ms * 1e-3) / 1e9 if launches else None
    roof = {
        "kernel": kernel,
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
        "traffic": recorded_traffic(kernel, wl.name),
        "launches": launches,
        "avg_us": avg_ms * 1e3,
        "algorithmic_bytes_per_launch": nbytes / max(launches, 1),
    }
    out = {
        "metric": "seconds per RHS to rel. residual 1e-6; V-cycle HBM GB/s vs peak",
        "value": sec32,
        "unit": "s/RHS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt32 / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 multigrid / c128 FGMRES",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.n), "nrhs": nrhs, "omega": wl.omega,
                   "levels": wl.levels, "cycle": "V(%d,%d)" % tuple(wl.nu), "alpha": wl.alpha,
                   "restart": wl.restart, "tol": wl.tol, "iters": it32, "relres_true": rel32},
        "fp64_plain": fp64,
        "roofline": roof,
        "kernel_split_one_solve": split or None,
        "vcycle_one_solve": vcycle_summary(split_bytes),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, it64, args.cpu_iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
