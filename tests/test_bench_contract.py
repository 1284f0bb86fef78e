"""The benchmark script's command-line contract, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_recorded_far_traffic_belongs_to_the_committed_kernel():
    # the HBM bytes reported in the roofline were measured on a specific far-kernel source; bench.py
    # reports null once the source changes, so a stale figure shows up here first
    sys.path.insert(0, ROOT)
    import bench

    assert bench.far_traffic("fp64") is not None and bench.far_traffic("mixed") is not None


def test_near_pair_count_equals_brute_force():
    """The roofline's far-pair count is M N less the pairs within the near radius; the k-d tree count
    behind it equals a direct count over every pair (small workload)."""
    import numpy as np

    sys.path.insert(0, ROOT)
    import bench
    import workload

    cfg = workload.build_config("small")
    x, y = cfg["surf"].x, cfg["targets"].y
    rnear = 6.0 * max(cfg["rho"]) * cfg["h"]
    d2 = ((y[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    assert bench.near_pair_count(cfg) == int((d2 <= rnear * rnear).sum())
    # 34 flops per far single-layer pair and 32 per double-layer pair
    assert bench.FAR_FLOPS_PER_PAIR_SLDL == 66
