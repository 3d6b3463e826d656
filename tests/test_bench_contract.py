"""Host-side checks of the benchmark script: the one-GPU contract, the
algorithmic flop count of an STGD run, and that the committed HBM counters
belong to the kernel sources in the tree (the bench line reports their
traffic only then)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_sgd_flops_counts_every_step():
    # per step 6 B k^2 (P_A, P_B and D) + 4 k^3 (G and O); the last batch of a pass is ragged
    k, batch, passes = 10, 4, 3
    full = 6.0 * batch * k * k + 4.0 * k ** 3
    last = 6.0 * 2 * k * k + 4.0 * k ** 3
    assert bench.sgd_flops(10, batch, k, passes) == passes * (2 * full + last)
    assert bench.sgd_flops(8, batch, k, 1) == 2 * full
    # the benchmark's run: 500 steps of B = 100 at k = 100, 50 passes
    assert bench.sgd_flops(50000, 100, 100, 50) == 2.5e11


def test_committed_counters_match_the_kernel_sources():
    sgd = json.load(open(os.path.join(ROOT, "profiles", "sgd_kernel_mmsb_large_counters.json")))
    assert sgd["kernel_sha256_16"] == bench.kernel_hash()
    assert bench.counters_traffic() == sgd["bytes_per_launch"] > sgd["algorithmic_bytes_per_launch"]
    wh = json.load(open(os.path.join(ROOT, "profiles", "whiten_kernel_counters.json")))
    assert wh["kernel_sha256_16"] == bench.kernel_hash(("spmm.hip",))
    for name in ("documents", "graph"):
        assert bench.whiten_traffic(name) == wh["workloads"][name]["bytes_per_launch"] > 0
