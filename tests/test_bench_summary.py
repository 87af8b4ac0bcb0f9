"""bench.py's counter and trace summarisers on small synthetic files (no
GPU): the 1 GiB calibration copy (the run's first copy, not a later larger
one) fixes the scale of each counter, only the last solve's dispatches of a
class (from the solve's one cycle-start norm, eh::k_gs<3>, on; copies
inside a solve do not cut it) are summed and divided by its timed launches
(a Gram-Schmidt pass is two dispatches), and the record carries the hash of
the kernel sources."""
import csv
import os

import bench


def _write(path, counter, rows):
    fields = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as fp:
        w = csv.DictWriter(fp, fieldnames=fields)
        w.writeheader()
        for i, (name, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": 256,
                        "Counter_Name": counter, "Counter_Value": val})


def test_pmc_summary_scales_by_the_copy_and_counts_timed_launches(tmp_path):
    gib_kib = (1 << 30) / 1024.0
    tune = ("void eh::k_fup<float, true, 2, 1>(eh::GArgs<float>, int)", 7777.0)   # set-up / tuning
    norm = ("void eh::k_gs<3>(long, int)", 0.0)                  # a solve's first cycle start
    fetch = [("__amd_rocclr_copyBuffer", gib_kib / 2),          # the counter reads half
             tune,
             ("__amd_rocclr_copyBuffer", gib_kib), norm,         # an earlier solve starts
             ("void eh::k_gs<4>(long, int)", 3000.0), tune,
             ("__amd_rocclr_copyBuffer", 2 * gib_kib), norm,     # the last solve starts (larger copy)
             ("void eh::k_gs<4>(long, int)", 1000.0), ("eh::k_reduce_partials(int)", 10.0),
             ("__amd_rocclr_copyBuffer", 3.0),                   # a copy inside the solve
             ("void eh::k_gs<2>(long, int)", 2000.0), ("eh::k_reduce_partials(int)", 10.0),
             ("void eh::k_fup<float, true, 2, 0>(eh::GArgs<float>, int)", 5000.0),
             ("void eh::k_gdense<float, 1>(eh::DenseArgs, eh::GArgs<float>)", 300.0)]
    write = [("__amd_rocclr_copyBuffer", gib_kib),
             tune,
             ("__amd_rocclr_copyBuffer", gib_kib), norm,
             ("void eh::k_gs<4>(long, int)", 3000.0), tune,
             ("__amd_rocclr_copyBuffer", 2 * gib_kib), norm,
             ("void eh::k_gs<4>(long, int)", 0.0), ("eh::k_reduce_partials(int)", 1.0),
             ("__amd_rocclr_copyBuffer", 3.0),
             ("void eh::k_gs<2>(long, int)", 500.0), ("eh::k_reduce_partials(int)", 1.0),
             ("void eh::k_fup<float, true, 2, 0>(eh::GArgs<float>, int)", 900.0),
             ("void eh::k_gdense<float, 1>(eh::DenseArgs, eh::GArgs<float>)", 100.0)]
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _write(f, "FETCH_SIZE", fetch)
    _write(w, "WRITE_SIZE", write)
    rec = bench.pmc_summary(str(f), str(w), "krylov", "test")
    assert rec["launches_fetch"] == 3 and rec["dispatches_fetch"] == 5
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    # the last solve's krylov class: its norm, two passes and their reductions (three timed launches)
    expect = ((0 + 1000 + 10 + 2000 + 10) / 3 * 2.0 + (0 + 0 + 1 + 500 + 1) / 3 * 1.0) * 1024.0
    assert abs(rec["traffic_bytes_per_launch"] - expect) < 1e-6
    assert rec["source_sha256"] == bench.sources_sha256(rec["source_files"])
    up = bench.pmc_summary(str(f), str(w), "fine_up", "test")
    assert up["launches_fetch"] == 1
    assert abs(up["traffic_bytes_per_launch"] - (5000 * 2.0 + 900) * 1024.0) < 1e-6
    vc = bench.pmc_summary(str(f), str(w), "vcycle", "test")
    assert vc["launches_fetch"] == 2 and vc["launches_write"] == 2
    assert abs(vc["traffic_bytes_per_launch"] - ((5000 + 300) * 2.0 + 900 + 100) / 2 * 1024.0) < 1e-6


def test_trace_summary_counts_the_last_solves(tmp_path):
    """Launch counts and mean durations over the last K solves of a kernel
    trace (each solve opens with its copy and its cycle-start norm; copies
    inside a solve do not cut it; earlier launches are ignored)."""
    import csv as _csv
    rows = [("__amd_rocclr_copyBuffer", 5), ("void eh::k_fup<float, true, 2, 1>(x)", 999),
            ("__amd_rocclr_copyBuffer", 5), ("void eh::k_gs<3>(long, int)", 2),
            ("void eh::k_fup<float, true, 2, 0>(x)", 20),
            ("void eh::k_gs<4>(long, int)", 30), ("eh::k_reduce_partials(int)", 4),
            ("__amd_rocclr_copyBuffer", 5), ("void eh::k_gs<3>(long, int)", 2),
            ("void eh::k_fup<float, false, 2, 0>(x)", 10),
            ("__amd_rocclr_copyBuffer", 5),
            ("void eh::k_fdown<float, true, 1>(x)", 12)]
    path = tmp_path / "trace.csv"
    with open(path, "w", newline="") as fp:
        wr = _csv.DictWriter(fp, fieldnames=["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        wr.writeheader()
        t = 1000
        for i, (name, us) in enumerate(rows):
            wr.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Start_Timestamp": t,
                         "End_Timestamp": t + us * 1000})
            t += us * 1000 + 500
    out = bench.trace_summary(str(path), 2)
    assert out["vcycle"]["launches"] == 3
    assert abs(out["vcycle"]["avg_us"] - (20 + 10 + 12) / 3) < 1e-9
    assert out["krylov"]["launches"] == 3 and abs(out["krylov"]["avg_us"] - (2 + 30 + 4 + 2) / 3) < 1e-9
    assert out["fine_up"]["launches"] == 1 and out["coarse_up"]["launches"] == 1


def test_recorded_traffic_matches_committed_record():
    """The committed fine up-leg record is found for its own workload while
    its sources are unchanged, and never for another workload or class."""
    import workloads as W
    t = bench.recorded_traffic("fine_up", W.config(4).name)
    assert t is None or t > 0
    assert bench.recorded_traffic("fine_up", W.config(2).name) is None
    assert bench.recorded_traffic("no_such_class", W.config(4).name) is None


def test_vcycle_summary_sums_bytes_and_time_of_the_multigrid_classes():
    """The V-cycle figure is total bytes over total duration of the multigrid
    classes only (not an average of their rates); the operator and Krylov
    classes count only in the share of the solve."""
    split = {"fine_down": (2.0, 6e9 * 2e-3), "coarse_up": (6.0, 1e9 * 6e-3), "dense": (1.0, 3e9 * 1e-3),
             "krylov": (4.0, 5e9 * 4e-3), "operator": (3.0, 4e9 * 3e-3)}
    v = bench.vcycle_summary(split)
    assert v["classes"] == ["fine_down", "coarse_up", "dense"]
    assert abs(v["achieved"] - (12e6 + 6e6 + 3e6) / 9e-3 / 1e9) < 0.05
    assert abs(v["frac"] - v["achieved"] / bench.HBM_PEAK_GBS) < 1e-5
    assert abs(v["share_of_solve"] - 9.0 / 16.0) < 1e-12
    assert bench.vcycle_summary({}) is None
