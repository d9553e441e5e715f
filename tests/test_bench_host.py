"""Host-side checks of bench.py (no GPU): the one-GPU refusal and the
committed profile of the dominant kernel."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_committed_profile_matches_the_kernel_sources():
    # the profile's counters (traffic, VALUBusy) are reported by bench.py only
    # while they describe the kernels as they are now
    vals = bench.profiled_values()
    assert vals, "profile missing or taken on other kernel sources"
    assert bench.profiled_traffic() > 0
    assert 0 < bench.profiled_float("valu_busy_pct") <= 100
    assert 0 < bench.profiled_float("valu_lane_activity_pct") <= 100
