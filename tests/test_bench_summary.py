"""bench.py's counter summariser on a small synthetic counter file (no GPU):
the 1 GiB calibration copy (the run's first copy, not a later larger one)
fixes the scale of each counter, dispatches of a
class are summed and divided by its timed launches (a Gram-Schmidt pass is
two dispatches), and the record carries the hash of the kernel sources."""
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
    fetch = [("__amd_rocclr_copyBuffer", gib_kib / 2),          # the counter reads half
             ("void eh::k_gs<4>(long, int)", 1000.0), ("eh::k_reduce_partials(int)", 10.0),
             ("void eh::k_gs<2>(long, int)", 2000.0), ("eh::k_reduce_partials(int)", 10.0),
             ("void eh::k_fup<float, true, 2, 0>(eh::GArgs<float>, int)", 5000.0),
             ("__amd_rocclr_copyBuffer", gib_kib)]                # a later, larger copy of the solver
    write = [("__amd_rocclr_copyBuffer", gib_kib),
             ("void eh::k_gs<4>(long, int)", 0.0), ("eh::k_reduce_partials(int)", 1.0),
             ("void eh::k_gs<2>(long, int)", 500.0), ("eh::k_reduce_partials(int)", 1.0),
             ("void eh::k_fup<float, true, 2, 0>(eh::GArgs<float>, int)", 900.0),
             ("__amd_rocclr_copyBuffer", 2 * gib_kib)]
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _write(f, "FETCH_SIZE", fetch)
    _write(w, "WRITE_SIZE", write)
    rec = bench.pmc_summary(str(f), str(w), "krylov", "test")
    assert rec["launches_fetch"] == 2 and rec["dispatches_fetch"] == 4
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    expect = ((1000 + 10 + 2000 + 10) / 2 * 2.0 + (0 + 1 + 500 + 1) / 2 * 1.0) * 1024.0
    assert abs(rec["traffic_bytes_per_launch"] - expect) < 1e-6
    assert rec["source_sha256"] == bench.sources_sha256(rec["source_files"])
    up = bench.pmc_summary(str(f), str(w), "fine_up", "test")
    assert up["launches_fetch"] == 1
    assert abs(up["traffic_bytes_per_launch"] - (5000 * 2.0 + 900) * 1024.0) < 1e-6


def test_recorded_traffic_matches_committed_record():
    """The committed Krylov record is found for its own workload while its
    sources are unchanged, and never for another workload or class."""
    import workloads as W
    t = bench.recorded_traffic("krylov", W.config(2).name)
    assert t is None or t > 0
    assert bench.recorded_traffic("krylov", W.config(4).name) is None
    assert bench.recorded_traffic("no_such_class", W.config(2).name) is None
