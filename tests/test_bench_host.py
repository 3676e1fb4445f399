"""Host-side checks of bench.py that need no GPU: the one-GPU guard and the
algorithmic byte counts its roofline divides by."""
import os
import subprocess
import sys

import bench
from paper_2609_29081_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_of_the_headline_grid():
    """a stage reads U^(k) (and U^n from the second stage on) and writes one
    state: 8/3 states per launch on average, 170.9 MB at 1000x500"""
    g, _ = W.shock_tube_2d(1000, 500)
    assert g.dof_sites == 2003001
    state = 8.0 * g.state_len
    assert state == 8.0 * 4 * 2003001
    alg = bench.algorithmic_bytes(g)
    assert abs(alg["stage2d"] - state * 8.0 / 3.0) <= 1.0
    assert abs(alg["stage2d"] - 170.9e6) < 0.05e6
