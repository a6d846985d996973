"""Host-side contract of bench.py (no GPU): the one-GPU refusal and the
rules by which the benchmark line reports counter-derived figures."""
import importlib.util
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_reported_only_for_the_profiled_configuration():
    b = _bench()
    # counters exist per workload and policy, in compensated mode only
    for kernel in ("k_far_mfma", "k_band_piece", "k_rt_walk"):
        assert b.measured_traffic(kernel, "C1", "fixed", 1) is None
        assert b.measured_traffic(kernel, "C5", "fixed", 0) is None
        assert b.measured_traffic(kernel, "C5", "learned", 2) is None
    assert b.measured_traffic("k_no_such_kernel", "C5", "learned", 1) is None


def test_probe_references_are_stored_for_the_bench_workloads():
    b = _bench()
    for name, k in (("C2", 24), ("C5", 32)):
        nodes, exact = b.load_probes(name)
        assert nodes.shape == (k,) and exact.shape == (k, 3)
        assert len(set(nodes.tolist())) == k and np.all(np.isfinite(exact))


def test_algorithmic_flops_counts_gauss_points_and_ray_work():
    b = _bench()
    # one pair of each Gauss rule: 1, 4 and 11 points at 26 flops each
    st = {"pairs_by_rule": [1, 1, 1, 0], "rt_hit_lines": 0}
    assert b.algorithmic_flops(st, 256) == 26.0 * 16
    # ray tracing: per pair 9 plus 7 per line of the N x M table, 156 per hit line
    st = {"pairs_by_rule": [0, 0, 0, 2], "rt_hit_lines": 3}
    assert b.algorithmic_flops(st, 256) == 2 * (9.0 + 7.0 * 256) + 156.0 * 3
