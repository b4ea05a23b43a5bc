"""Host-side logic of the benchmark's measurement (no GPU): turning
rocprofv3 FETCH_SIZE / WRITE_SIZE runs into HBM bytes per launch scaled by a
copy of known size, and withholding those bytes once the kernel's source (or
a shared header) has changed since the counters were taken."""
import argparse
import csv
import os
import shutil
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Kernel_Name", "Counter_Name", "Counter_Value"]


def _run_dir(path, rows):
    os.makedirs(path)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        wr = csv.DictWriter(fh, fieldnames=FIELDS)
        wr.writeheader()
        for name, counter, value in rows:
            wr.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})
    return path


def _tree(tmp):
    src = os.path.join(ROOT, "paper_1711_02976_amd", "csrc")
    dst = os.path.join(tmp, "paper_1711_02976_amd", "csrc")
    os.makedirs(dst)
    for f in ("nearfield.hip", "m2l_rot.hip", "common.h", "fmm.h"):
        shutil.copy(os.path.join(src, f), dst)
    os.makedirs(os.path.join(tmp, "profiles"))
    return dst


def test_counters_scaled_by_the_copy_and_withheld_when_stale(tmp_path, monkeypatch):
    tmp = str(tmp_path)
    csrc = _tree(tmp)
    monkeypatch.setattr(bench, "ROOT", tmp)
    k = "rpy::k_p2p_mfma<true, 0>(int4 const*, ...)"
    f = _run_dir(os.path.join(tmp, "f"), [(k, "FETCH_SIZE", 100.0), (k, "FETCH_SIZE", 300.0),
                                         ("rpy::k_m2m<16>(int)", "FETCH_SIZE", 5.0)])
    w = _run_dir(os.path.join(tmp, "w"), [(k, "WRITE_SIZE", 40.0), (k, "WRITE_SIZE", 40.0),
                                         ("rpy::k_m2m<16>(int)", "WRITE_SIZE", 1.0)])
    # a 1 MiB copy whose fetch counter reads half the bytes and write counter all of them
    cf = _run_dir(os.path.join(tmp, "cf"), [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0)])
    cw = _run_dir(os.path.join(tmp, "cw"), [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0)])
    args = argparse.Namespace(pmc_summary=[f, w, cf, cw], copy_probe=1, workload="cube-15M")
    assert bench.pmc_summary(args) == 0
    key = "p2p_mc:cube-15M:mixed"
    assert bench.traffic_for("nearfield.hip", key) == round(200.0 * 1024 * 2.0) + round(40.0 * 1024 * 1.0)
    assert bench.traffic_for("nearfield.hip", "p2p:cube-15M:mixed") is None  # no such kernel in the run
    # an edit of the kernel file or of a shared header makes the figure stale
    with open(os.path.join(csrc, "fmm.h"), "a") as fh:
        fh.write("\n")
    assert bench.traffic_for("nearfield.hip", key) is None
