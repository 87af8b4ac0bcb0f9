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


def oracle_iterations(wl):
    """The oracle's own iteration counts on this workload, from the record
    tests/golden/make_oracle_iterations.py wrote (None when there is none)."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_iterations_{wl.name}.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("workload") != wl.name:
        return None
    return rec


_CPU = {}


def _cpu_sample(q):
    """n FGMRES iterations of the oracle on source q (forked worker)."""
    from oracle.fgmres import fgmres
    H, M, b, wl, n = _CPU["H"], _CPU["M"], _CPU["b"], _CPU["wl"], _CPU["n"]
    t0 = time.perf_counter()
    res = fgmres(lambda x: H @ x, M, b[q % b.shape[0]], restart=wl.restart, tol=wl.tol, maxit=n)
    return (time.perf_counter() - t0) / max(res.iters, 1)


def cpu_baseline(wl, n_iters, procs, gpu_fp64_iters=None):
    """The oracle (NumPy/SciPy FP64, one thread per process) on the same
    workload: setup once (not timed), then `n_iters` FGMRES iterations
    timed in one process, and again in `procs` processes forked after the
    setup, each on its own source (right-hand sides are independent: the
    RHS-parallel throughput of the host).  Seconds per RHS = seconds per
    iteration x the oracle's own iteration count on this workload (mean over
    its sources, tests/golden/oracle_iterations_*.json), or the GPU's FP64
    count where the oracle has no record (labelled)."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle.elastic import ElasticSystem
    from oracle.precond import BlockAcoustic

    rec = oracle_iterations(wl)
    if rec is not None:
        iters, iters_src = rec["iters_mean"], (f"the oracle's own count, mean over its {len(rec['sources'])} "
                                               f"sources ({rec['iters_min']}..{rec['iters_max']}), recorded by "
                                               f"{rec['script']}")
    else:
        iters, iters_src = gpu_fp64_iters, "no oracle record for this workload: the GPU's FP64 iteration count"
    with threadpool_limits(1):
        t0 = time.perf_counter()
        s = ElasticSystem(wl.n, wl.h, wl.vp, wl.vs, wl.rho, wl.omega, wl.abc_width, wl.abc_sides)
        _CPU.update(H=s.H(), M=BlockAcoustic(s, alpha=wl.alpha, solver="mg", levels=wl.levels, cycle="V",
                                             nu=wl.nu, damping=wl.damping, intergrid=wl.intergrid),
                    b=W.point_source_rhs(wl.n, wl.h, wl.sources), wl=wl, n=n_iters)
        setup = time.perf_counter() - t0
        log(f"cpu baseline: oracle setup {setup:.1f} s")
        t1 = _cpu_sample(0)
        log(f"cpu baseline: one process {t1:.3f} s per iteration")
        tp = None
        if procs > 1:
            with mp.get_context("fork").Pool(procs) as pool:
                tp = max(pool.map(_cpu_sample, range(procs), chunksize=1))
            log(f"cpu baseline: {procs} processes {tp:.3f} s per iteration each")
    _CPU.clear()
    if iters is None:
        return None
    single = t1 * iters
    par = tp * iters / procs if tp else single
    return {
        "value": par,
        "unit": "s/RHS",
        "cores": procs if tp else 1,
        "kind": "oracle",
        "sample": (f"the oracle (NumPy/SciPy FP64 sparse V-cycles, MGS FGMRES, splu coarsest; setup "
                   f"{setup:.0f} s not timed) on the same workload ({wl.name}): {n_iters} FGMRES iterations "
                   f"timed in one process ({t1:.3f} s/iteration) and in {procs} processes at once, one "
                   f"source each, one thread each ({tp if tp else t1:.3f} s/iteration, the slowest); "
                   f"extrapolated to {iters:.2f} iterations per RHS ({iters_src}); value = RHS-parallel "
                   f"throughput over {procs} processes"),
        "single_process_s_per_rhs": single,
        "iterations_per_rhs": iters,
        "extrapolated": True,
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
def _gfine(*modes):
    """Kernel names of the fine-level sweeps of the given modes (per point,
    and plane-staged in 3D, which has modes 1, 2 and 5)."""
    return (tuple(f"eh::k_gfine<{t}, {k}, {d}, {m}>" for m in modes for t in ("float", "double")
                  for k in (0, 1, 2) for d in (2, 3))
            + tuple(f"eh::k_gfine3_lds<{t}, {k}, {m}>" for m in modes if m in (1, 2, 5)
                    for t in ("float", "double") for k in (0, 1, 2)))


CLASS_KERNELS = {
    "krylov": (("eh::k_gs<", "eh::k_reduce_partials", "eh::k_xupdate<"), ("eh::k_gs<", "eh::k_xupdate<")),
    "fine_down": (("eh::k_fdown<float, true", "eh::k_fdown<double, true"), None),
    "fine_up": (("eh::k_fup<float, true", "eh::k_fup<double, true"), None),
    "coarse_down": (("eh::k_fdown<float, false", "eh::k_fdown<double, false"), None),
    "coarse_up": (("eh::k_fup<float, false", "eh::k_fup<double, false"), None),
    "coarse": (("eh::k_gstencil<", "eh::k_gstencil3_lds<"), None),
    "fine_sweep": (_gfine(1), None),
    "fine_resid": (_gfine(2), None),
    "fine_first": (_gfine(0, 4, 5), None),
    "restrict": (("eh::k_gtransfer<float, 2, true>", "eh::k_gtransfer<float, 3, true>",
                  "eh::k_gtransfer<double, 2, true>", "eh::k_gtransfer<double, 3, true>",
                  "eh::k_grestrict3_lds<"), None),
    "prolong": (("eh::k_gtransfer<float, 2, false>", "eh::k_gtransfer<float, 3, false>",
                 "eh::k_gtransfer<double, 2, false>", "eh::k_gtransfer<double, 3, false>",
                 "eh::k_gprolong3_lds<"), None),
    "operator": (("eh::k_op2_lds<", "eh::k_op3_lds<"), None),
    "distribute": (("eh::k_distribute<",), None),
    "couple": (("eh::k_gcouple<",), None),
    "dense": (("eh::k_gdense<", "eh::k_bt_fpart<", "eh::k_bt_chain<"), None),
    # every timed multigrid kernel: the V-cycles of the three (four) blocks
    "vcycle": (("eh::k_fdown<", "eh::k_fup<", "eh::k_gdense<", "eh::k_gstencil<", "eh::k_gfine<",
                "eh::k_gtransfer<", "eh::k_bt_fpart<", "eh::k_bt_chain<", "eh::k_gfine3_lds<",
                "eh::k_gstencil3_lds<", "eh::k_grestrict3_lds<", "eh::k_gprolong3_lds<"), None),
}
DEFAULT_SOURCES = ["paper_2411_15897_amd/csrc/eh_fused_kernels.h", "paper_2411_15897_amd/csrc/eh_group_kernels.h",
                   "paper_2411_15897_amd/csrc/eh_mg_kernels.h", "paper_2411_15897_amd/csrc/eh_op_kernels.h",
                   "paper_2411_15897_amd/csrc/eh_common.h"]
_FINE3 = DEFAULT_SOURCES + ["paper_2411_15897_amd/csrc/eh_fine3_kernels.h"]
_STENCIL3 = DEFAULT_SOURCES + ["paper_2411_15897_amd/csrc/eh_stencil3_kernels.h"]
_TRANSFER3 = DEFAULT_SOURCES + ["paper_2411_15897_amd/csrc/eh_transfer3_kernels.h"]
CLASS_SOURCES = {
    "krylov": ["paper_2411_15897_amd/csrc/eh_krylov_kernels.h", "paper_2411_15897_amd/csrc/eh_common.h"],
    "fine_sweep": _FINE3, "fine_resid": _FINE3, "fine_first": _FINE3, "coarse": _STENCIL3,
    "restrict": _TRANSFER3, "prolong": _TRANSFER3,
    "dense": DEFAULT_SOURCES + ["paper_2411_15897_amd/csrc/eh_coarse_kernels.h"],
    "vcycle": _FINE3 + ["paper_2411_15897_amd/csrc/eh_stencil3_kernels.h",
                        "paper_2411_15897_amd/csrc/eh_transfer3_kernels.h",
                        "paper_2411_15897_amd/csrc/eh_coarse_kernels.h"],
}




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


def pmc_summary(fetch_csv, write_csv, kernel, workload, config=None):
    """HBM traffic per timed launch of a kernel class from a FETCH_SIZE and a
    WRITE_SIZE rocprofv3 counter run (KiB per dispatch), each scaled by what
    the same counter reads for the 1 GiB calibration copy of the same run
    (the run's first copy dispatch: it precedes the solver's own copies).
    Only the run's last solve counts: the dispatches from its SOLVE_MARK
    dispatch on, so set-up and tuning launches do not enter."""
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
        marks = [int(r["Dispatch_Id"]) for r in rows if SOLVE_MARK in r["Kernel_Name"]]
        if not marks:
            raise SystemExit(f"bench.py: {path} holds no {SOLVE_MARK} dispatch (no solve)")
        last = max(marks)                               # start of the last solve
        cls = [r for r in rows if int(r["Dispatch_Id"]) >= last and any(m in r["Kernel_Name"] for m in members)]
        nlaunch = sum(1 for r in cls if any(m in r["Kernel_Name"] for m in leads))
        kib = sum(float(r["Counter_Value"]) for r in cls) / max(nlaunch, 1)
        rec[f"{tag}_kib_per_launch_raw"] = kib
        rec[f"copy_{tag}_kib"] = ref
        rec[f"{tag}_scale"] = scale
        rec[f"launches_{tag}"] = nlaunch
        rec[f"dispatches_{tag}"] = len(cls)
        total += kib * scale * 1024.0
    rec["copy_reference"] = "torch copy of 1 GiB (__amd_rocclr_copyBuffer) in the same runs"
    rec["launches_counted"] = "the dispatches of the run's last solve (from its first Gram-Schmidt norm on)"
    rec["traffic_bytes_per_launch"] = total
    rec["source_files"] = CLASS_SOURCES.get(kernel, DEFAULT_SOURCES)
    rec["source_sha256"] = sources_sha256(rec["source_files"])
    run = "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp64 --copy-calibration"
    if config is not None:
        run += f" --config {config}"
    fdir, wdir = os.path.dirname(fetch_csv), os.path.dirname(write_csv)
    rec["commands"] = [
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {fdir} -o run -- {run}",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {wdir} -o run -- {run}",
        f"python3 bench.py --roofline-kernel {kernel} --pmc-summary {fetch_csv} {write_csv}"
        + (f" --config {config}" if config is not None else ""),
    ]
    return rec


# Each solve's first cycle start, and nothing else in a benchmark run, takes
# the norm of b with the Gram-Schmidt kernel's mode 3: its dispatches mark
# where the solves begin in a trace or a counter run.
SOLVE_MARK = "eh::k_gs<3>"


def trace_summary(trace_csv, solves):
    """Per kernel class (and the vcycle group): launches and average
    duration over the last `solves` solves of a rocprofv3 --kernel-trace
    run of this script with --no-fp64 --no-cpu-baseline (its last solves
    are the event-timed ones; each begins at its SOLVE_MARK dispatch)."""
    import csv
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Dispatch_Id"]))
    starts = [i for i, r in enumerate(rows) if SOLVE_MARK in r["Kernel_Name"]]
    if solves < 1 or len(starts) < solves:
        raise SystemExit(f"bench.py: {trace_csv} holds {len(starts)} solves ({SOLVE_MARK} dispatches), "
                         f"fewer than --steps {solves}")
    tail = rows[starts[-solves]:]
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
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--restart", type=int, default=None)
    ap.add_argument("--roofline-kernel", default=None,
                    help="kernel class (or the group vcycle: every multigrid kernel) for the roofline figure "
                         "(default: fine_up, the fused fine up leg, in 2D; fine_sweep, the fine-level "
                         "Jacobi sweep, in 3D)")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--cpu-procs", type=int, default=None,
                    help="processes of the RHS-parallel CPU baseline (default: min(16, host threads))")
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
        wl_ = W.config(args.config)
        kernel_ = args.roofline_kernel or ("fine_up" if len(wl_.n) == 2 else "fine_sweep")
        print(json.dumps(pmc_summary(*args.pmc_summary, kernel_, wl_.name, args.config), indent=1))
        return
    if args.gpus != 1:
        print("bench.py: this solver runs on one GPU only; several GPUs would each take a share of "
              "the sources, with one all-reduce of the gradient at the end",
              file=sys.stderr)
        sys.exit(2)

    import workloads as W

    wl = W.config(args.config)
    if args.levels:
        wl.levels = args.levels
    if args.alpha is not None:
        wl.alpha = args.alpha
    if args.restart:
        wl.restart = args.restart
    b_host = W.point_source_rhs(wl.n, wl.h, wl.sources)
    nrhs = b_host.shape[0]

    # the CPU baseline first: its worker processes are forked before this
    # process touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        procs = args.cpu_procs or max(1, min(16, os.cpu_count() or 1))
        cpu = cpu_baseline(wl, args.cpu_iters, procs)

    import numpy as np
    import torch

    from paper_2411_15897_amd import ElasticHelmholtz

    dev = torch.device("cuda:0")
    b = torch.from_numpy(b_host).to(dev)

    def make(prec):
        return ElasticHelmholtz(wl.n, wl.h, wl.vp, wl.vs, wl.rho, wl.omega, levels=wl.levels,
                                nu=wl.nu, damping=wl.damping, alpha=wl.alpha, mg_precision=prec,
                                restart=wl.restart, abc_width=wl.abc_width,
                                abc_sides=wl.abc_sides, intergrid=wl.intergrid)

    all_infos = {"c64": [], "c128": []}

    def timed(solver, steps, warmup, kernel=None):
        x = None
        for w in range(warmup):
            x, info = solver.solve(b, tol=wl.tol, maxit=5000)
            all_infos["c64"].append(info)
            log(f"warmup {w}: iters {[i['iters'] for i in info]}")
        classes = timer_classes(kernel) if kernel else []
        for k in classes:
            solver.timer_read(k)               # drop anything recorded before
        if classes:
            solver.timer_enable(classes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for k in range(steps):
            x, info = solver.solve(b, tol=wl.tol, maxit=5000)
            infos.append(info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        all_infos["c64"].extend(infos)
        kt = None
        if classes:
            reads = [solver.timer_read(k) for k in classes]
            kt = tuple(sum(r[i] for r in reads) for i in range(3))
        solver.timer_enable([])
        log(f"timed {steps} solves in {dt:.3f} s, iters {[[i['iters'] for i in inf] for inf in infos]}")
        return dt, infos, kt, x

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)       # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"workload {wl.name}: n={wl.n} nrhs={nrhs} omega={wl.omega:.4f} levels={wl.levels} alpha={wl.alpha}")
    t_setup = time.perf_counter()
    s32 = make(32)
    torch.cuda.synchronize()
    log(f"setup (complex64 multigrid) {time.perf_counter() - t_setup:.2f} s")
    kernel = args.roofline_kernel or ("fine_up" if len(wl.n) == 2 else "fine_sweep")
    split = {}
    split_bytes = {}
    # one untimed solve with every kernel class event-timed: the split of
    # the solve over the classes
    from paper_2411_15897_amd._native import KERNEL_CLASSES
    s32.timer_enable(list(KERNEL_CLASSES))
    _, info = s32.solve(b, tol=wl.tol, maxit=5000)
    all_infos["c64"].append(info)
    for k in KERNEL_CLASSES:
        n_, ms_, by_ = s32.timer_read(k)
        if n_:
            split[k] = {"launches": n_, "ms": round(ms_, 3),
                        "GB_s": round(by_ / (ms_ * 1e-3) / 1e9, 1)}
            split_bytes[k] = (ms_, by_)
    s32.timer_enable([])
    log(f"per-class split of one solve: {json.dumps(split)}")
    # value: the solve as it runs (Arnoldi steps replayed from HIP graphs)
    dt32, inf32, _, x32 = timed(s32, args.steps, args.warmup, None)
    # roofline: the same K solves again with every launch of the roofline
    # class bracketed by HIP events on the solver's stream (plain launches;
    # the kernels are the same, only the launch path differs), and of the
    # whole V-cycle group
    _, _, kt, _ = timed(s32, args.steps, 0, kernel)
    kt_v = None
    if kernel != "vcycle":
        _, _, kt_v, _ = timed(s32, 1, 0, "vcycle")
    s32.close()
    sec32 = dt32 / (args.steps * nrhs)
    it32 = [i["iters"] for i in inf32[-1]]

    fp64 = None
    if not args.no_fp64:
        # the plain form: complex128 multigrid, every source solved on its
        # own, one after the other
        s64 = make(64)
        _, info = s64.solve(b[0:1], tol=wl.tol, maxit=5000)          # warm-up (tuning, graphs)
        all_infos["c128"].append(info)
        x64 = torch.empty_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inf64 = []
        for q in range(nrhs):
            _, info = s64.solve(b[q:q + 1], tol=wl.tol, maxit=5000, x=x64[q:q + 1])
            inf64.append(info[0])
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        all_infos["c128"].append(inf64)
        s64.close()
        errs = [(torch.linalg.vector_norm(x32[q] - x64[q]) / torch.linalg.vector_norm(x64[q])).item()
                for q in range(nrhs)]
        fp64 = {"form": f"complex128 multigrid, the {nrhs} sources solved one at a time (all timed)",
                "s_per_rhs": dt64 / nrhs, "iters": [i["iters"] for i in inf64],
                "relres_true_max": max(i["relres_true"] for i in inf64),
                "value_speedup": (dt64 / nrhs) / sec32,
                "x32_vs_x64_rel_err": {"max": max(errs), "min": min(errs), "per_source": errs}}
        log(f"fp64 single-RHS solves: {dt64 / nrhs:.4f} s per RHS, iters {fp64['iters']}, "
            f"max |x32 - x64|/|x64| {max(errs):.2e}")

    # validity: every right-hand side of every solve converged below tol
    flat = [i for k in all_infos for inf in all_infos[k] for i in (inf if isinstance(inf, list) else [inf])]
    valid = all(i["converged"] and i["relres_true"] < wl.tol for i in flat)

    def roof_of(kt_, name):
        launches, ms, nbytes = kt_
        avg_ms = ms / max(launches, 1)
        achieved = (nbytes / max(launches, 1)) / (avg_ms * 1e-3) / 1e9 if launches else None
        return {
            "kernel": name,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": recorded_traffic(name, wl.name),
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
        "valid": valid,
        "config": {"workload": wl.name, "grid": list(wl.n), "nrhs": nrhs, "batched": True, "omega": wl.omega,
                   "levels": wl.levels, "cycle": "V(%d,%d)" % tuple(wl.nu), "alpha": wl.alpha,
                   "intergrid": wl.intergrid, "restart": wl.restart, "tol": wl.tol, "iters": it32,
                   "relres_true_max": max(i["relres_true"] for inf in inf32 for i in inf)},
        "fp64_plain": fp64,
        "roofline": roof_of(kt, kernel),
        "roofline_vcycle_group": roof_of(kt_v, "vcycle") if kt_v else None,
        "kernel_split_one_solve": split or None,
        "vcycle_one_solve": vcycle_summary(split_bytes),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    if not valid:
        log("bench.py: a right-hand side did not converge below the tolerance; the line is invalid")
        sys.exit(3)


if __name__ == "__main__":
    main()
