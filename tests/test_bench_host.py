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
    import bench

    # 250 walked points, 300 lookups, 29 hits, 3 factors
    assert bench.work_bytes(250, 300, 29, 3) == 250 * 36 + 300 * 8 + 29 * 36 + 3 * (48 + 344)


def test_roofline_bound_is_the_higher_fraction():
    sys.path.insert(0, ROOT)
    import bench

    tk = {"tile_kernel_ms": 2.0, "reduce_ms": 0.01}
    B = int(0.5 * bench.HBM_PEAK * 2e-3)                 # half of peak over 2 ms
    r = bench.make_roofline(B, 2 * B, 10, tk, None, "k")
    assert r["bound"] == "hbm" and abs(r["frac"] - 0.5) < 1e-12 and r["unit"] == "GB/s"
    assert abs(r["hbm_frac_every_point"] - 1.0) < 1e-12 and r["valu_issue_frac"] is None
    # 70 % VALU issue: wave instructions x 64 lanes over the lane peak
    valu = 0.7 * bench.VALU_PEAK * 2e-3 / 64
    r = bench.make_roofline(B, 2 * B, 10, tk, {"valu_insts": valu, "traffic_bytes": 1e9, "l2_hit_rate": 0.4,
                                               "source": "x"}, "k")
    assert r["bound"] == "alu" and abs(r["frac"] - 0.7) < 1e-12 and r["unit"] == "TOP/s"
    assert abs(r["hbm_frac"] - 0.5) < 1e-12 and abs(r["dram_frac"] - 1e9 / 2e-3 / bench.HBM_PEAK) < 1e-12
    assert r["frac"] <= 1.0
    # walked-work bytes above peak (shared sources re-read from caches): the counters'
    # DRAM fraction decides against the VALU fraction
    r = bench.make_roofline(4 * B, 4 * B, 10, tk, {"valu_insts": valu, "traffic_bytes": 0.4 * bench.HBM_PEAK * 2e-3,
                                                   "l2_hit_rate": 0.4, "source": "x"}, "k")
    assert r["hbm_frac"] > 1.0 and r["bound"] == "alu" and abs(r["frac"] - 0.7) < 1e-12
    r = bench.make_roofline(4 * B, 4 * B, 10, tk, {"valu_insts": valu, "traffic_bytes": 0.9 * bench.HBM_PEAK * 2e-3,
                                                   "l2_hit_rate": 0.4, "source": "x"}, "k")
    assert r["bound"] == "hbm"


def test_measured_counters_follow_sources_and_launch(tmp_path):
    """The bench reports counter figures only while the kernel sources' hash and
    the launch shape match the profile summary it reads."""
    sys.path.insert(0, ROOT)
    import bench

    launch = {"block_threads": 128, "tile_points": 8192, "grid_blocks": 2048, "tile_order": 1}
    body = ("launch: block 128 tile 8192 grid 2048 order 1\ntraffic_bytes_per_launch: 1.5e+10 (note)\n"
            "l2_hit_rate: 0.4200\nvalu_insts_per_dispatch: 1.3e+09\n")
    good = tmp_path / "good.txt"
    good.write_text("# summary\nkernel_sources_sha256: %s\n" % bench.kernel_sources_sha256() + body)
    c = bench.measured_counters(str(good), launch)
    assert c["traffic_bytes"] == 1.5e10 and c["l2_hit_rate"] == 0.42 and c["valu_insts"] == 1.3e9
    assert bench.measured_counters(str(good), dict(launch, tile_points=4096)) is None
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_sources_sha256: %s\n" % ("0" * 64) + body)
    assert bench.measured_counters(str(stale), launch) is None
    assert bench.measured_counters(str(tmp_path / "missing.txt"), launch) is None
