"""Benchmark: source points linearized per second (e, H, b), batched vs plain.

Default workload: the global submap batch -- 500 synthetic submaps of
50k-300k points (log-uniform), 0.5 m voxels, 5,000 submap-to-submap factors
(submap i against i +- 3..7) -- linearized in compensated FP32.  A step is
one full linearization of the whole batch with everything resident in HBM:
the poses are a device buffer before timing starts and the device-pointer
entry point leaves e/H/b and the inlier counts on the device (pose staging,
tile kernel, factor reduction).  The host-buffer entry point (one captured
hipGraph: upload poses, the same kernels, download results) is timed beside
it and reported as ``host_buffers``; the plain per-factor path is compared
with that one, since both hand over host buffers.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
B_POINT = 36               # mu (12) + C (24), FP32, per (factor, source point)
B_KEY = 8                  # one hash slot per (point, level)
B_HIT = 36                 # voxel mean (12) + covariance (24) per hit
B_FACTOR = 48 + 344        # pose in + e/H/b/inliers out per factor
COPY_BYTES = 1 << 30       # calibration copy for the memory counters


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name, n_submaps):
    import synth
    t = time.time()
    if name == "global":
        cfg = synth.config3(n_submaps=n_submaps)
        desc = {"workload": "global submap batch", "submaps": n_submaps, "factors": len(cfg["factors"]),
                "points_per_submap": "50k-300k log-uniform", "voxel_m": 0.5, "levels": 1}
    elif name == "odometry":
        cfg = synth.config2()
        desc = {"workload": "odometry batch", "factors": 20, "points_per_frame": cfg["sources"][0].n,
                "voxel_m": [0.25, 0.5, 1.0, 2.0], "levels": 4}
    elif name == "single":
        cfg = synth.config1()
        desc = {"workload": "single factor", "factors": 1, "source_points": 5000, "target_points": 20000,
                "voxel_m": 0.5, "levels": 1}
    else:
        raise SystemExit("unknown workload " + name)
    log("generated %s in %.1f s" % (name, time.time() - t))
    return cfg, desc


def algorithmic_bytes(cfg, inliers):
    pts = sum(cfg["sources"][s].n for (s, _) in cfg["factors"])
    L = inliers.shape[1]
    hits = int(inliers.sum())
    return pts * B_POINT + pts * L * B_KEY + hits * B_HIT + len(cfg["factors"]) * B_FACTOR, pts, hits


def cpu_baseline(cfg, batch_out, budget_s=10.0):
    """FP64 oracle on a time-bounded sample of the factors, one factor per host core.

    Factors are taken in a seeded random order; no new factor starts after
    ``budget_s`` seconds.  The rate is source points of the finished factors over
    the wall time, with the target voxel maps built beforehand (outside the timing).
    """
    import oracle
    oracle.build()
    fac = cfg["factors"]
    res = cfg["resolutions"]
    cores = len(os.sched_getaffinity(0))
    order = [int(f) for f in np.random.default_rng(0).permutation(len(fac))]
    # candidate sample: enough work for the budget at a generous per-core rate
    cand, acc = [], 0
    for f in order:
        cand.append(f)
        acc += cfg["sources"][fac[f][0]].n
        if acc > 5e7 * cores * budget_s:
            break
    targets = sorted({fac[f][1] for f in cand})

    def build_map(t):
        tg = cfg["targets"][t]
        return t, oracle.VoxelMap(tg.xyz64(), tg.cov64(), res)

    with ThreadPoolExecutor(cores) as ex:
        maps = dict(ex.map(build_map, targets))
    factors = {}
    for f in cand:
        s, t = fac[f]
        src = cfg["sources"][s]
        factors[f] = oracle.Factor(src.xyz64(), src.cov64(), maps[t], viewpoint=cfg["target_viewpoints"][f])

    t0 = time.perf_counter()
    deadline = t0 + budget_s

    def run(f):
        if time.perf_counter() > deadline:
            return f, None
        return f, factors[f].linearize(cfg["poses"][f])

    with ThreadPoolExecutor(cores) as ex:
        results = {f: r for f, r in ex.map(run, cand) if r is not None}
    dt = time.perf_counter() - t0
    pts = sum(cfg["sources"][fac[f][0]].n for f in results)
    # single-thread rate on the first factors of the same sample (about 3 s)
    t1, pts1 = time.perf_counter(), 0
    for f in cand:
        factors[f].linearize(cfg["poses"][f])
        pts1 += cfg["sources"][fac[f][0]].n
        if time.perf_counter() - t1 > 3.0:
            break
    single = pts1 / (time.perf_counter() - t1)
    # parity of the device results on the same sample: relative errors e / H (Frobenius) / b.
    # Every factor above the tolerance, plus the 32 worst below it, is re-checked with the
    # face-band rule (a point within 1e-5 m of a voxel face may take either neighbouring
    # voxel; the oracle then scores the device's choice).
    parity = {"factors": len(results)}
    if batch_out is not None:
        from oracle.parity import expected_with_device_keys, rel_err
        e, H, b, batch = batch_out
        raw = {f: {"e": rel_err(e[f], r["e"]), "H": rel_err(H[f], r["H"]), "b": rel_err(b[f], r["b"])}
               for f, r in results.items()}
        worst_first = sorted(raw, key=lambda f: -max(raw[f].values()))
        over = [f for f in worst_first if max(raw[f].values()) > 1e-5]
        recheck = worst_first[:len(over) + 32]
        final = dict(raw)
        for f in recheck:
            kd, fd = batch.correspondences(cfg["poses"][f], f)
            ee, HH, bb, _ = expected_with_device_keys(factors[f], cfg["poses"][f], kd, fd)
            final[f] = {"e": rel_err(e[f], ee), "H": rel_err(H[f], HH), "b": rel_err(b[f], bb)}
        mx = lambda d: {k: max(v[k] for v in d.values()) for k in ("e", "H", "b")} if d else None
        parity.update({"max_raw": mx(raw), "raw_over_1e-5": len(over), "face_band_rechecked": len(recheck),
                       "max_after_face_band": mx(final),
                       "max_rechecked_after_face_band": mx({f: final[f] for f in recheck})})
    return {"value": pts / dt, "unit": "source points/s", "cores": cores, "kind": "oracle",
            "single_thread_value": single,
            "sample": "%d of %d factors (%d source points) in %.1f s, FP64 C oracle, one factor per thread" % (
                len(results), len(fac), pts, dt)}, parity


KERNEL_SOURCES = ("paper_2407_10344_amd/csrc/vg_factor.hip", "paper_2407_10344_amd/csrc/vg_device.h",
                  "paper_2407_10344_amd/csrc/vg_internal.h")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_summary_path(workload, submaps, precision):
    tag = "global_%dsubmaps" % submaps if workload == "global" else workload
    return os.path.join(ROOT, "profiles", "k_tiles_lin_%s_%s.txt" % (precision, tag))


def read_profile_summary(path):
    out = {}
    if not os.path.exists(path):
        return out
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#", "|")):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def measured_traffic(path, launch):
    """HBM bytes per tile-kernel launch from the committed counter summary, or None
    when the summary is missing, was taken with another launch shape, or the
    kernel sources changed since."""
    p = read_profile_summary(path)
    try:
        if p.get("kernel_sources_sha256") != kernel_sources_sha256():
            return None
        if p.get("launch") != "block %d tile %d grid %d order %d" % (
                launch["block_threads"], launch["tile_points"], launch["grid_blocks"], launch["tile_order"]):
            return None
        return float(p["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _csvs(d, suffix):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def summarize_profiles(kt_dir, fetch_dir, write_dir, command, tile_points, tile_order, workload, warmup):
    """Text summary of one rocprofv3 kernel-trace run and two counter runs
    (FETCH_SIZE, WRITE_SIZE) of ``bench.py --profile-steps``.  The counters are
    scaled by what they read for the calibration kernels of known size that the
    profile run ends with (a 1 GiB fill: write; a 1 GiB sum: read)."""
    import csv
    tile_prefix = "void vg::k_tiles<0, 0,"
    stats = []
    for f in _csvs(kt_dir, "_kernel_stats.csv"):
        stats += list(csv.DictReader(open(f)))
    tile = [r for r in stats if r["Name"].startswith(tile_prefix)]
    if len(tile) != 1:
        raise SystemExit("expected one tile-kernel row in the kernel stats, found %d" % len(tile))
    tile = tile[0]

    # steady state: tile-kernel dispatches after the warm-up steps, from the kernel trace
    durs = []
    for f in _csvs(kt_dir, "_kernel_trace.csv"):
        for r in csv.DictReader(open(f)):
            if r["Kernel_Name"].startswith(tile_prefix):
                durs.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    durs = [d for _, d in sorted(durs)][warmup:]
    shapes = set()

    def counters(d, name):
        per = {}
        for f in _csvs(d, "_counter_collection.csv"):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == name:
                    per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
                    if r["Kernel_Name"].startswith(tile_prefix):
                        shapes.add((int(r["Workgroup_Size"]), int(r["Grid_Size"]) // int(r["Workgroup_Size"])))
        return per

    fetch = counters(fetch_dir, "FETCH_SIZE")
    write = counters(write_dir, "WRITE_SIZE")

    def pick(per, pred):
        ks = [k for k in per if pred(k)]
        if len(ks) != 1:
            raise SystemExit("expected one matching kernel, found %d" % len(ks))
        v = per[ks[0]]
        return sum(v) / len(v), len(v)

    f_tile, nf = pick(fetch, lambda k: k.startswith(tile_prefix))
    w_tile, nw = pick(write, lambda k: k.startswith(tile_prefix))
    f_red = pick(fetch, lambda k: k.startswith("void vg::k_reduce<0, 0>"))[0]
    w_red = pick(write, lambda k: k.startswith("void vg::k_reduce<0, 0>"))[0]
    sums = [max(v) for k, v in fetch.items() if "reduce_kernel" in k]
    fills = [max(v) for k, v in write.items() if "FillFunctor<float>" in k]
    if not sums or not fills:
        raise SystemExit("calibration kernels not found in the counter runs")
    if len(shapes) != 1:
        raise SystemExit("tile kernel launched with several shapes: %s" % sorted(shapes))
    (block, grid), = shapes
    kib = COPY_BYTES / 1024.0
    f_scale = kib / max(sums)
    w_scale = kib / max(fills)
    traffic = (f_tile * f_scale + w_tile * w_scale) * 1024.0
    lines = [
        "# rocprofv3 summary: tile kernel k_tiles<lin, fp32c> (linearize, compensated FP32), %s" % workload,
        "#",
        "# commands (from /tmp, TMPDIR=/tmp, REPO = the repository root):",
    ] + ["#   " + c for c in command] + [
        "#",
        "kernel: %s" % tile["Name"].split("(")[0],
        "launch: block %d tile %d grid %d order %d" % (block, tile_points, grid, tile_order),
        "kernel_sources_sha256: %s" % kernel_sources_sha256(),
        "tile_kernel_calls: %s" % tile["Calls"],
        "tile_kernel_avg_ns: %.0f" % float(tile["AverageNs"]),
        "tile_kernel_min_ns: %s" % tile["MinNs"],
        "tile_kernel_max_ns: %s" % tile["MaxNs"],
        "tile_kernel_steady_avg_ns: %.0f (%d dispatches after %d warm-up steps)" % (
            sum(durs) / max(len(durs), 1), len(durs), warmup),
        "fetch_size_kib_per_dispatch: %.1f" % f_tile,
        "write_size_kib_per_dispatch: %.1f" % w_tile,
        "reduce_fetch_kib_per_dispatch: %.1f" % f_red,
        "reduce_write_kib_per_dispatch: %.1f" % w_red,
        "calibration_sum_fetch_kib: %.1f" % max(sums),
        "calibration_fill_write_kib: %.1f" % max(fills),
        "fetch_scale: %.4f" % f_scale,
        "write_scale: %.4f" % w_scale,
        "traffic_bytes_per_launch: %.6e" % traffic,
        "counter_dispatches: %d fetch, %d write" % (nf, nw),
        "",
        "top kernels of the kernel-trace run (total time):",
        "| calls | avg us | total ms | % | kernel |",
        "|---|---|---|---|---|",
    ]
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in stats[:10]:
        lines.append("| %s | %.1f | %.2f | %.1f | %s |" % (r["Calls"], float(r["AverageNs"]) / 1e3,
                                                       float(r["TotalDurationNs"]) / 1e6,
                                                       float(r["Percentage"]), r["Name"][:110]))
    return "\n".join(lines) + "\n"


def summarize_counters(dirs, command):
    """Mean per dispatch of each counter of the tile kernel k_tiles<lin, fp32c>."""
    import csv
    from collections import defaultdict
    agg = defaultdict(list)
    for d in dirs:
        for f in _csvs(d, "_counter_collection.csv"):
            for r in csv.DictReader(open(f)):
                if r["Kernel_Name"].startswith("void vg::k_tiles<0, 0,"):
                    agg[r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["# rocprofv3 counters of the tile kernel k_tiles<lin, fp32c> (mean per dispatch)", "#"]
    lines += ["#   " + c for c in command] + ["#"]
    for k in sorted(agg):
        lines.append("%s: %.6e (%d dispatches)" % (k, sum(agg[k]) / len(agg[k]), len(agg[k])))
    return "\n".join(lines) + "\n"


def bench_preprocess(args, r=0.25, k=10):
    """Frame preprocessing: one raw 128-ring frame (host FP64) -> downsampled cloud
    with k-NN, covariances and normals on the device; a step is one frame."""
    import torch
    import synth
    from paper_2407_10344_amd import vgicp
    pts, sensor = synth.raw_frame()
    ctx = vgicp.Context(0)
    for _ in range(args.warmup):
        vgicp.Cloud(ctx, pts, r, k, sensor).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        c = vgicp.Cloud(ctx, pts, r, k, sensor)
        m = c.n
        c.close()
    dt = (time.perf_counter() - t0) / args.steps
    out = {"metric": "raw LiDAR points preprocessed/sec (downsample + exact k-NN + covariances + normals)",
           "value": len(pts) / dt, "unit": "raw points/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "frame preprocessing", "rings": 128, "azimuth_steps": 1024,
                      "raw_points": len(pts), "downsampled_points": m, "voxel_m": r, "k": k,
                      "includes": "host-to-device upload of the raw frame and every allocation"}}
    print(json.dumps(out), flush=True)
    ctx.close()


def time_steps(batch, poses, steps, warmup):
    """Seconds per linearize step of a batch, two ways.

    device: poses already in device memory, the device-pointer entry point
    (pose staging, tile kernel, reduction; e/H/b and inlier counts stay on the
    device).  host: the host-buffer entry point, which adds the pose upload and
    the result download.  Returns (dt_device, dt_host, host results, whether
    both entry points gave identical bits)."""
    import torch
    d_poses = torch.tensor(np.ascontiguousarray(poses), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        out, inl_d = batch.linearize_async(d_poses)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out, inl_d = batch.linearize_async(d_poses)
    torch.cuda.synchronize()
    dt_dev = (time.perf_counter() - t0) / steps
    for _ in range(warmup):
        res = batch.linearize(poses)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = batch.linearize(poses)
    torch.cuda.synchronize()
    dt_host = (time.perf_counter() - t0) / steps
    e, H, b, inl = res
    o = out.cpu().numpy()
    same = bool(np.array_equal(o[:, 0], e) and np.array_equal(o[:, 1:37].reshape(-1, 6, 6), H)
                and np.array_equal(o[:, 37:43], b) and np.array_equal(inl_d.cpu().numpy(), inl))
    return dt_dev, dt_host, res, same


def bench_local(args, r=0.25, k=10, res=(0.25, 0.5, 1.0)):
    """Local-mapping batch: 15 raw frames preprocessed on the device, 105
    all-to-all factors with surface validation; a step is one linearization of
    the batch (poses resident, one upload / download)."""
    import torch
    import synth
    from paper_2407_10344_amd import vgicp
    d = synth.local_mapping()
    ctx = vgicp.Context(0)
    t0 = time.perf_counter()
    clouds = [vgicp.Cloud(ctx, p, r, k, np.zeros(3)) for p in d["raw"]]
    srcs = [vgicp.Source.from_cloud(ctx, c) for c in clouds]
    maps = [vgicp.VoxelMap.from_cloud(ctx, c, list(res)) for c in clouds]
    torch.cuda.synchronize()
    prep_ms = (time.perf_counter() - t0) * 1e3 / len(clouds)
    pairs = d["pairs"]
    shape = {"block": args.block, "tile": args.tile, "blocks_per_cu": args.bpc, "tile_order": args.tile_order}
    batch = vgicp.FactorBatch(ctx, [srcs[i] for i, _ in pairs], [maps[j] for _, j in pairs],
                              viewpoints=np.zeros((len(pairs), 3)), precision=args.precision, validation=True,
                              use_graph=True, lane_kahan=args.lane_kahan, **shape)
    poses = vgicp.poses12(np.array(d["rel_est"]))
    if not args.no_tune and not any(shape.values()):
        batch.tune(poses, reps=3)
    info = batch.info()
    dt, dt_host, (e, H, b, inl), same = time_steps(batch, poses, args.steps, args.warmup)
    log("device-resident %.3f ms/step, host buffers %.3f ms/step, identical results: %s"
        % (dt * 1e3, dt_host * 1e3, same))
    pts = sum(c.n for c in (clouds[i] for i, _ in pairs))
    hits = int(inl.sum())
    L = inl.shape[1]
    B_alg = pts * B_POINT + pts * L * B_KEY + hits * B_HIT + len(pairs) * B_FACTOR
    tk = batch.time_kernels(poses, reps=20)
    plain = vgicp.FactorBatch(ctx, [srcs[i] for i, _ in pairs], [maps[j] for _, j in pairs],
                              viewpoints=np.zeros((len(pairs), 3)), precision=args.precision, validation=True,
                              use_graph=False, plain=True, block=info["block_threads"], tile=info["tile_points"])
    plain.linearize(poses)
    t0 = time.perf_counter()
    for _ in range(5):
        plain.linearize(poses)
    plain_dt = (time.perf_counter() - t0) / 5
    plain.close()
    out = {"metric": "source points linearized/sec (e,H,b), batched vs plain, at rel. err <=1e-5",
           "value": pts / dt, "unit": "source points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp32c": "f32", "fp32": "f32", "fp64": "f64"}[args.precision], "data": "synthetic",
           "config": {"workload": "local-mapping batch", "frames": len(clouds), "factors": len(pairs),
                      "voxel_m": list(res), "levels": L, "surface_validation": True, "precision": args.precision,
                      "total_source_points": pts, "inlier_pairs": hits, "launch": info,
                      "preprocess_ms_per_frame": prep_ms},
           "host_buffers": {"value": pts / dt_host, "ms_per_step": dt_host * 1e3,
                            "includes": "pose upload and result download"},
           "plain": {"value": pts / plain_dt, "unit": "source points/s", "batched_speedup": plain_dt / dt_host},
           "roofline": {"bound": "hbm", "achieved": B_alg / (tk["tile_kernel_ms"] * 1e-3) / 1e9,
                        "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": B_alg / (tk["tile_kernel_ms"] * 1e-3) / HBM_PEAK, "traffic": None,
                        "kernel_ms": tk["tile_kernel_ms"], "reduce_ms": tk["reduce_ms"], "call_ms": tk["call_ms"],
                        "algorithmic_bytes": B_alg}}
    print(json.dumps(out), flush=True)
    batch.close()
    for x in srcs + maps + clouds:
        x.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="global", choices=["global", "odometry", "single", "preprocess", "local"])
    ap.add_argument("--submaps", type=int, default=500)
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp32", "fp64"])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0: library default / tuned)")
    ap.add_argument("--tile", type=int, default=0, help="source points per tile (0: default / tuned)")
    ap.add_argument("--bpc", type=int, default=0, help="persistent workgroups per CU (0: default / tuned)")
    ap.add_argument("--tile-order", type=int, default=0,
                    help="1: contiguous tile range per XCD, 2: tiles dealt round-robin to XCDs (0: default / tuned)")
    ap.add_argument("--lane-kahan", action="store_true", help="Kahan-compensated FP32 sums inside each lane")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run --warmup + this many batched steps (for profilers), print no JSON")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("KT_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write the text summary of three rocprofv3 runs of --profile-steps and exit")
    ap.add_argument("--profile-command", action="append", default=[],
                    help="command line recorded in the summary (repeatable)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_DIR",
                    help="print the mean per dispatch of every counter of the tile kernel in rocprofv3 --pmc runs")
    args = ap.parse_args()
    if args.summarize_counters:
        sys.stdout.write(summarize_counters(args.summarize_counters, args.profile_command))
        return
    if args.summarize_profiles:
        tag = "global submap batch, %d submaps" % args.submaps if args.workload == "global" else args.workload
        sys.stdout.write(summarize_profiles(*args.summarize_profiles, args.profile_command, args.tile,
                                            args.tile_order or 1, tag, args.warmup))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_10344_amd import vgicp

    if args.workload == "preprocess":
        bench_preprocess(args)
        return
    if args.workload == "local":
        bench_local(args)
        return
    cfg, desc = make_workload(args.workload, args.submaps)
    ctx = vgicp.Context(0)
    t = time.time()
    shape = {"block": args.block, "tile": args.tile, "blocks_per_cu": args.bpc, "tile_order": args.tile_order}
    maps, srcs, batch = vgicp.build_workload(ctx, cfg, precision=args.precision, use_graph=True,
                                             lane_kahan=args.lane_kahan, **shape)
    torch.cuda.synchronize()
    log("device maps/sources/batch built in %.1f s" % (time.time() - t))
    poses = vgicp.poses12(np.array(cfg["poses"]))
    info = batch.info()
    if not args.no_tune and args.profile_steps == 0 and not any(shape.values()):
        t = time.time()
        chosen = batch.tune(poses, reps=2)
        info = batch.info()
        log("autotuned %s in %.1f s" % (chosen, time.time() - t))

    if args.profile_steps:
        for _ in range(args.warmup + args.profile_steps):
            batch.linearize(poses)
        torch.cuda.synchronize()
        # kernels of known traffic, to scale the memory counters: a fill that
        # writes COPY_BYTES and a reduction that reads them
        src_t = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        total = src_t.sum()
        torch.cuda.synchronize()
        log("profile run done: %d + %d warm-up linearize steps; calibration: fill (write) and sum (read) of %d bytes, %s"
            % (args.profile_steps, args.warmup, COPY_BYTES, float(total)))
        return

    dt, dt_host, (e, H, b, inl), same = time_steps(batch, poses, args.steps, args.warmup)
    log("device-resident %.3f ms/step, host buffers %.3f ms/step, identical results: %s"
        % (dt * 1e3, dt_host * 1e3, same))
    B_alg, pts, hits = algorithmic_bytes(cfg, inl)
    value = pts / dt

    # dominant kernel time, HIP events on the library's stream
    tk = batch.time_kernels(poses, reps=max(3, min(args.steps, 20)))
    achieved = B_alg / (tk["tile_kernel_ms"] * 1e-3)

    # plain per-factor path (one upload, launch, download and sync per factor)
    plain_rate = None
    if args.plain_steps > 0:
        _, _, plain = vgicp.build_workload(ctx, cfg, precision=args.precision, use_graph=False, plain=True,
                                           block=info["block_threads"], tile=info["tile_points"],
                                           tile_order=info["tile_order"])
        plain.linearize(poses)
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            ep, Hp, bp, _ = plain.linearize(poses)
        plain_dt = (time.perf_counter() - t0) / args.plain_steps
        plain_rate = pts / plain_dt
        same = bool(np.array_equal(ep, e) and np.array_equal(Hp, H) and np.array_equal(bp, b))
        plain.close()
        log("plain per-factor: %.1f ms/step, identical results: %s" % (plain_dt * 1e3, same))

    prof_path = profile_summary_path(args.workload, args.submaps, args.precision)
    traffic = measured_traffic(prof_path, info)
    log("measured traffic per launch: %s (%s)" % (traffic, os.path.relpath(prof_path, ROOT)))

    cpu, parity = (None, None)
    if not args.no_cpu:
        cpu, parity = cpu_baseline(cfg, (e, H, b, batch))
        log("cpu baseline", cpu, "parity on sample", parity)

    dtype = {"fp32c": "f32", "fp32": "f32", "fp64": "f64"}[args.precision]
    out = {
        "metric": "source points linearized/sec (e,H,b), batched vs plain, at rel. err <=1e-5",
        "value": value,
        "unit": "source points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": dict(desc, precision=args.precision, lane_kahan=bool(args.lane_kahan),
                       total_source_points=pts, inlier_pairs=hits,
                       hit_rate=hits / max(pts, 1), launch=info),
        "host_buffers": {"value": pts / dt_host, "ms_per_step": dt_host * 1e3,
                         "includes": "pose upload and result download"},
        "plain": None if plain_rate is None else {"value": plain_rate, "unit": "source points/s",
                                                  "batched_speedup": (pts / dt_host) / plain_rate},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": traffic,
                     "dram_frac": None if traffic is None else traffic / (tk["tile_kernel_ms"] * 1e-3) / HBM_PEAK,
                     "kernel": "k_tiles<lin,%s>" % args.precision, "kernel_ms": tk["tile_kernel_ms"],
                     "reduce_ms": tk["reduce_ms"], "algorithmic_bytes": B_alg},
        "cpu_baseline": cpu,
        "parity_sample": parity,
    }
    print(json.dumps(out), flush=True)
    batch.close()


if __name__ == "__main__":
    main()
