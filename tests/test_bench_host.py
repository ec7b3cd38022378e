"""Host-side checks of bench.py that need no GPU."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_accounting():
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench

    class C:
        def __init__(self, n):
            self.n = n

    cfg = {"sources": [C(100), C(50)], "factors": [(0, 1), (1, 0), (0, 0)]}
    inl = np.array([[10, 5], [0, 0], [7, 7]])
    B, pts, hits = bench.algorithmic_bytes(cfg, inl)
    assert pts == 250 and hits == 29
    assert B == 250 * 36 + 250 * 2 * 8 + 29 * 36 + 3 * (48 + 344)
