"""Host-side parts of bench.py: the one-GPU refusal and the algorithmic work
it divides by the kernel time (CPU)."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_lu_flops_is_the_complex_lu_count():
    # complex LU: N^3/3 complex multiply-adds (8 real flops each), then the
    # port block: P right-hand sides through N^2 complex multiply-adds
    N = np.array([3, 769], np.int64)
    got = bench.lu_flops(N, 2)
    assert np.allclose(got, 8.0 / 3.0 * N.astype(np.float64) ** 3 + 8.0 * 2 * N.astype(np.float64) ** 2)
    assert abs(bench.lu_flops(np.array([3]), 1)[0] - (72.0 + 72.0)) < 1e-9
