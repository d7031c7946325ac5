"""Host logic of bench.py (no GPU): the one-GPU refusal and the rule that
counter figures are reported only for the executor source they were taken
on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_counter_figures_follow_the_kernel_source():
    d = bench.counters_from_profile(bench.kernel_source_hash())
    if d:  # taken on the current executor source: every figure is there
        assert d["hbm_bytes_per_step"] > 0
        assert d["l2_atomic_requests_per_step"] > 0
        assert 0 < d["l2_hit_fraction"] < 1
    assert bench.counters_from_profile("0" * 40) == {}
