"""Host-side parts of the benchmark's contract: one GPU only (a request for
more exits with a message and a nonzero status before touching a GPU), and
the stored HBM-counter figures are keyed by the kernel sources they were
taken from, so the benchmark can tell whether they still apply."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU only" in r.stderr and r.stdout.strip() == ""


def test_traffic_figures_are_keyed_by_kernel_source():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as fh:
        data = json.load(fh)
    workload = "lattice9_n128_a360_b192_batch64"
    entry = data[workload]["k_vjp_lin"]
    assert entry["bytes_per_launch"] > 0 and len(entry["kernel_source"]) == 16
    # a figure applies exactly when it was taken from the current sources
    expect = entry["bytes_per_launch"] if entry["kernel_source"] == h else None
    assert bench.traffic_from_profile("k_vjp_lin", workload) == expect
