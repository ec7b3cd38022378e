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


def test_measured_traffic_follows_sources_and_launch(tmp_path):
    """The bench reports counter traffic only while the kernel sources' hash and
    the launch shape match the profile summary it reads."""
    sys.path.insert(0, ROOT)
    import bench

    launch = {"block_threads": 128, "tile_points": 8192, "grid_blocks": 2048, "tile_order": 1}
    good = tmp_path / "good.txt"
    good.write_text("# summary\nkernel_sources_sha256: %s\nlaunch: block 128 tile 8192 grid 2048 order 1\n"
                    "traffic_bytes_per_launch: 1.5e+10\n" % bench.kernel_sources_sha256())
    assert bench.measured_traffic(str(good), launch) == 1.5e10
    assert bench.measured_traffic(str(good), dict(launch, tile_points=4096)) is None
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_sources_sha256: %s\nlaunch: block 128 tile 8192 grid 2048 order 1\n"
                     "traffic_bytes_per_launch: 1.5e+10\n" % ("0" * 64))
    assert bench.measured_traffic(str(stale), launch) is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt"), launch) is None
