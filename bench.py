"""Benchmark: source points linearized per second (e, H, b), batched vs plain.

Default workload: the global submap batch -- 500 synthetic submaps of
50k-300k points (log-uniform), 0.5 m voxels, 5,000 submap-to-submap factors
(submap i against i +- 3..7) -- linearized in FP32 with compensated
accumulation, one captured hipGraph per step (upload poses, tile kernel,
factor reduction, download results).  A step is one full linearization of the
whole batch; inputs are resident in HBM before timing starts.

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
    # parity of the device results on the same sample: relative errors e / H (Frobenius) / b;
    # factors above the tolerance are re-checked with the face-band rule (a point within
    # 1e-5 m of a voxel face may take either neighbouring voxel)
    worst = {"e": 0.0, "H": 0.0, "b": 0.0, "factors": len(results), "face_band_rechecked": 0}
    if batch_out is not None:
        from oracle.parity import expected_with_device_keys, rel_err
        e, H, b, batch = batch_out
        for f, r in results.items():
            errs = {"e": rel_err(e[f], r["e"]), "H": rel_err(H[f], r["H"]), "b": rel_err(b[f], r["b"])}
            if max(errs.values()) > 1e-5:
                kd, fd = batch.correspondences(cfg["poses"][f], f)
                ee, HH, bb, _ = expected_with_device_keys(factors[f], cfg["poses"][f], kd, fd)
                errs = {"e": rel_err(e[f], ee), "H": rel_err(H[f], HH), "b": rel_err(b[f], bb)}
                worst["face_band_rechecked"] += 1
            for k in ("e", "H", "b"):
                worst[k] = max(worst[k], errs[k])
    return {"value": pts / dt, "unit": "source points/s", "cores": cores, "kind": "oracle",
            "sample": "%d of %d factors (%d source points) in %.1f s, FP64 C oracle, one factor per thread" % (
                len(results), len(fac), pts, dt)}, worst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="global", choices=["global", "odometry", "single"])
    ap.add_argument("--submaps", type=int, default=500)
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp32", "fp64"])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0: library default / tuned)")
    ap.add_argument("--tile", type=int, default=0, help="source points per tile (0: default / tuned)")
    ap.add_argument("--bpc", type=int, default=0, help="persistent workgroups per CU (0: default / tuned)")
    ap.add_argument("--lane-kahan", action="store_true", help="Kahan-compensated FP32 sums inside each lane")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many batched steps (for profilers), print nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_10344_amd import vgicp

    cfg, desc = make_workload(args.workload, args.submaps)
    ctx = vgicp.Context(0)
    t = time.time()
    shape = {"block": args.block, "tile": args.tile, "blocks_per_cu": args.bpc}
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
        for _ in range(args.profile_steps):
            batch.linearize(poses)
        torch.cuda.synchronize()
        # kernels of known traffic, to scale the memory counters: a fill that
        # writes COPY_BYTES and a reduction that reads them
        src_t = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        total = src_t.sum()
        torch.cuda.synchronize()
        log("profile run done: %d linearize steps; calibration: fill (write) and sum (read) of %d bytes, %s"
            % (args.profile_steps, COPY_BYTES, float(total)))
        return

    for _ in range(args.warmup):
        e, H, b, inl = batch.linearize(poses)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e, H, b, inl = batch.linearize(poses)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    B_alg, pts, hits = algorithmic_bytes(cfg, inl)
    value = pts / dt

    # dominant kernel time, HIP events on the library's stream
    tk = batch.time_kernels(poses, reps=max(3, min(args.steps, 20)))
    achieved = B_alg / (tk["tile_kernel_ms"] * 1e-3)

    # plain per-factor path (one upload, launch, download and sync per factor)
    plain_rate = None
    if args.plain_steps > 0:
        _, _, plain = vgicp.build_workload(ctx, cfg, precision=args.precision, use_graph=False, plain=True,
                                           block=info["block_threads"], tile=info["tile_points"])
        plain.linearize(poses)
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            ep, Hp, bp, _ = plain.linearize(poses)
        plain_dt = (time.perf_counter() - t0) / args.plain_steps
        plain_rate = pts / plain_dt
        same = bool(np.array_equal(ep, e) and np.array_equal(Hp, H) and np.array_equal(bp, b))
        plain.close()
        log("plain per-factor: %.1f ms/step, identical results: %s" % (plain_dt * 1e3, same))

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
        "plain": None if plain_rate is None else {"value": plain_rate, "unit": "source points/s",
                                                  "batched_speedup": value / plain_rate},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": None,
                     "kernel": "k_tiles<lin,%s>" % args.precision, "kernel_ms": tk["tile_kernel_ms"],
                     "reduce_ms": tk["reduce_ms"], "algorithmic_bytes": B_alg},
        "cpu_baseline": cpu,
        "parity_sample": parity,
    }
    print(json.dumps(out), flush=True)
    batch.close()


if __name__ == "__main__":
    main()
