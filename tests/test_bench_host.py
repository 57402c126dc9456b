"""Host-side logic of the benchmark script (no GPU): the one-GPU contract and
the HBM-traffic summary built from rocprofv3 counter files."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _counters(path, counter, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for i, (kernel, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter,
                        "Counter_Value": value})


def test_traffic_summary_scales_counters_by_the_copy_calibration(tmp_path):
    """A copy of COPY_BYTES whose FETCH_SIZE reads half its size and whose
    WRITE_SIZE reads its size gives factors 2 and 1; a kernel's bytes per
    launch are its mean counter (KiB) times 1024 times the factor."""
    d = str(tmp_path)
    kib = bench.COPY_BYTES / 1024.0
    copy = "__amd_rocclr_copyBuffer"
    jeig = "void k_jeig<float, 64, 1024, 1>(cx<float> const*, int)"
    _counters(os.path.join(d, "copy_fetch", "run_counter_collection.csv"), "FETCH_SIZE",
              [(copy, kib / 2), ("k_other(int)", 1.0)])
    _counters(os.path.join(d, "copy_write", "run_counter_collection.csv"), "WRITE_SIZE",
              [(copy, kib)])
    _counters(os.path.join(d, "fetch", "run_counter_collection.csv"), "FETCH_SIZE",
              [(jeig, 100.0), (jeig, 300.0)])
    _counters(os.path.join(d, "write", "run_counter_collection.csv"), "WRITE_SIZE",
              [(jeig, 50.0), (jeig, 50.0)])
    bench.summarize_pmc(d)
    out = json.load(open(os.path.join(d, "traffic.json")))
    cal = out["calibration"]
    assert cal["copy_kernel"] == copy
    assert abs(cal["fetch_factor"] - 2.0) < 1e-12 and abs(cal["write_factor"] - 1.0) < 1e-12
    k = out["kernels"]["k_jeig"]
    assert k["launches"] == 2
    assert abs(k["fetch_bytes_per_launch"] - 200.0 * 1024 * 2) < 1e-6
    assert abs(k["write_bytes_per_launch"] - 50.0 * 1024) < 1e-6
    assert abs(k["hbm_bytes_per_launch"] - (409600.0 + 51200.0)) < 1e-6
    assert out["source_sha256"] == bench.source_digest()
