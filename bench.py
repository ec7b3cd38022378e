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

Roofline: the algorithmic bytes are charged for the work the kernel does --
36 B per walked source point (chunks whose bounds cannot reach a target voxel
are culled before their points are read), 8 B per table lookup, 36 B per voxel
hit, 392 B per factor -- from the exact per-factor counts the kernels export,
over the tile kernel's average time from HIP events on the library stream.
Beside it: the same bytes with every source point charged, the unique
footprint of one launch (sources + voxel maps), and, from the committed
rocprofv3 summary of the same kernel source and launch shape, the DRAM
traffic, the L2 hit rate and the VALU issue fraction; ``bound`` is whichever
of the HBM fraction and the VALU issue fraction is higher.

Other workloads: ``--workload odometry|single|local|preprocess`` and the
differentiation (``diff``: 64 factors x 100k points, forward + backward) and
precision-stress (``precision``: 4 factors x 1M points 10 km from the origin,
a 10-iteration Levenberg-Marquardt loop per precision mode) batches.

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
CLOCK_HZ = 2.4e9           # MI355X peak engine clock
SIMDS = 256 * 4            # compute units x SIMDs per unit
VALU_PEAK = SIMDS * 16 * CLOCK_HZ   # lane operations/s: a wave64 VALU instruction issues over 4 cycles
B_POINT = 36               # mu (12) + C (24), FP32, per (factor, source point)
B_KEY = 8                  # one hash slot per (point, level)
B_HIT = 36                 # voxel mean (12) + covariance (24) per hit
B_FACTOR = 48 + 344        # pose in + e/H/b/inliers out per factor
COPY_BYTES = 1 << 30       # calibration copy for the memory counters
# launch shapes the autotuner measured on an MI355X, per batch signature (read
# by the library; a batch without an entry is tuned and its shape appended)
TUNE_CACHE = os.path.join(ROOT, "paper_2407_10344_amd", "tuned_shapes.jsonl")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _save_clouds(path, cfg):
    """The generated global batch as plain arrays (np.savez, no pickled objects)."""
    arr = {"resolutions": np.asarray(cfg["resolutions"]), "factors": np.asarray(cfg["factors"], dtype=np.int64),
           "poses": np.asarray(cfg["poses"]), "poses_true": np.asarray(cfg["poses_true"]),
           "target_viewpoints": np.asarray(cfg["target_viewpoints"]), "n_clouds": np.array(len(cfg["sources"]))}
    for i, c in enumerate(cfg["sources"]):
        arr["c%d_origin" % i] = c.origin
        arr["c%d_off" % i] = c.off32
        arr["c%d_cov" % i] = c.cov32
        arr["c%d_nrm" % i] = c.nrm32
        arr["c%d_vp" % i] = c.viewpoint
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arr)
    os.replace(tmp, path)


def _load_clouds(path):
    import synth
    z = np.load(path, allow_pickle=False)
    clouds = [synth.Cloud(origin=z["c%d_origin" % i], off32=z["c%d_off" % i], cov32=z["c%d_cov" % i],
                          nrm32=z["c%d_nrm" % i], viewpoint=z["c%d_vp" % i]) for i in range(int(z["n_clouds"]))]
    return {"name": "global submap batch", "targets": clouds, "sources": clouds,
            "resolutions": z["resolutions"].tolist(), "factors": [tuple(int(v) for v in f) for f in z["factors"]],
            "poses": list(z["poses"]), "poses_true": list(z["poses_true"]),
            "target_viewpoints": list(z["target_viewpoints"])}


def make_workload(name, n_submaps, cache=None):
    import synth
    t = time.time()
    if name == "global":
        if cache and os.path.exists(cache):
            cfg = _load_clouds(cache)
        else:
            cfg = synth.config3(n_submaps=n_submaps)
            if cache:
                _save_clouds(cache, cfg)
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


def cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


PARITY_KEYS = ("e", "H", "b", "H_ww", "H_wv", "H_vv", "H_scaled")


def cpu_baseline(cfg, batch_out, budget_s=8.0, runs=5):
    """FP64 oracle on a sample of the factors, one factor per host core.

    Factors are taken in a seeded random order; in a first pass no new factor
    starts after ``budget_s`` seconds, and the factors that finished form the
    sample, which is then timed ``runs - 1`` more times: the rate is its source
    points over the median wall time, with the target voxel maps built
    beforehand (outside the timing).
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
    times = [time.perf_counter() - t0]
    sample = sorted(results)
    for _ in range(runs - 1):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda f: factors[f].linearize(cfg["poses"][f]), sample))
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    pts = sum(cfg["sources"][fac[f][0]].n for f in results)
    # single-thread rate on the first factors of the same sample (about 3 s)
    t1, pts1 = time.perf_counter(), 0
    for f in cand:
        factors[f].linearize(cfg["poses"][f])
        pts1 += cfg["sources"][fac[f][0]].n
        if time.perf_counter() - t1 > 3.0:
            break
    single = pts1 / (time.perf_counter() - t1)
    # parity of the device results on the same sample: relative errors of e, H, b and of
    # the blocks of H.  Every factor above the tolerance, plus the 32 worst below it, is
    # re-checked with the face-band rule (a point within 1e-5 m of a voxel face may take
    # either neighbouring voxel; the oracle then scores the device's choice), and there
    # the halves of b are also bounded against the scale of their summands.
    parity = {"factors": len(results)}
    if batch_out is not None:
        from oracle.parity import ASSERTED, block_errors, expected_with_device_keys, rel_err
        e, H, b, batch = batch_out

        def errs_of(f, ee, HH, bb, scale=None):
            d = {"e": rel_err(e[f], ee), "H": rel_err(H[f], HH), "b": rel_err(b[f], bb)}
            d.update(block_errors(H[f], b[f], HH, bb, scale))
            return d

        raw = {f: errs_of(f, r["e"], r["H"], r["b"]) for f, r in results.items()}
        worst_first = sorted(raw, key=lambda f: -max(raw[f][k] for k in PARITY_KEYS))
        over = [f for f in worst_first if max(raw[f][k] for k in PARITY_KEYS) > 1e-5]
        recheck = worst_first[:len(over) + 32]
        final = dict(raw)
        for f in recheck:
            kd, fd = batch.correspondences(cfg["poses"][f], f)
            ee, HH, bb, _ = expected_with_device_keys(factors[f], cfg["poses"][f], kd, fd)
            final[f] = errs_of(f, ee, HH, bb, factors[f].gradient_scale(cfg["poses"][f]))

        def mx(d, keys):
            return {k: max(v[k] for v in d.values()) for k in keys} if d else None

        parity.update({"max_raw": mx(raw, PARITY_KEYS), "raw_over_1e-5": len(over),
                       "face_band_rechecked": len(recheck), "max_after_face_band": mx(final, PARITY_KEYS),
                       "max_rechecked_after_face_band": mx({f: final[f] for f in recheck}, ASSERTED)})
    return {"value": pts / dt, "unit": "source points/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(), "single_thread_value": single, "runs": runs,
            "sample": "%d of %d factors (%d source points), median of %d runs of %.2f-%.2f s, FP64 C oracle, "
                      "one factor per thread" % (len(results), len(fac), pts, runs, min(times), max(times))}, parity


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


def measured_counters(path, launch):
    """Counter figures of the tile kernel from the committed rocprofv3 summary
    (DRAM bytes per launch, L2 hit rate, VALU instructions per launch), or None
    when the summary is missing, was taken with another launch shape, or the
    kernel sources changed since."""
    p = read_profile_summary(path)
    if p.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    if p.get("launch") != "block %d tile %d grid %d order %d" % (
            launch["block_threads"], launch["tile_points"], launch["grid_blocks"], launch["tile_order"]):
        return None

    def num(k):
        try:
            return float(p[k].split()[0])
        except (KeyError, ValueError, IndexError):
            return None

    return {"traffic_bytes": num("traffic_bytes_per_launch"), "l2_hit_rate": num("l2_hit_rate"),
            "valu_insts": num("valu_insts_per_dispatch"), "source": os.path.relpath(path, ROOT)}


def _csvs(d, suffix):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


TILE_PREFIX = "void vg::k_tiles<0, 0,"


def _counter_means(dirs):
    """{kernel name: {counter: (mean per dispatch, dispatches)}} over rocprofv3 --pmc runs."""
    import csv
    per = {}
    for d in dirs:
        for f in _csvs(d, "_counter_collection.csv"):
            for r in csv.DictReader(open(f)):
                per.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(
                    (float(r["Counter_Value"]), int(r["Workgroup_Size"]), int(r["Grid_Size"])))
    return per


def summarize_profiles(kt_dir, pmc_dirs, command, tile_points, tile_order, workload, warmup, block=0):
    """Text summary of one rocprofv3 kernel-trace run and several counter runs of
    ``bench.py --profile-steps``.  Memory counters are read against the
    calibration kernels of known traffic the profile run ends with: a fill that
    writes COPY_BYTES, a sum that streams them, and a gather of 64-byte rows in
    random order (COPY_BYTES of rows plus the 8-byte indices).  FETCH_SIZE
    charges every read request 64 bytes: the streaming sum reads half its bytes
    (its requests are 128 bytes), and the random 64-byte rows read about twice
    theirs (a miss moves a whole 128-byte line, as two counted requests).  So
    the tile kernel's DRAM reads lie between FETCH_SIZE (every request 64 bytes)
    and twice it (every request 128 bytes)."""
    import csv
    prefix = TILE_PREFIX + (" %d," % block if block else "")
    stats = []
    for f in _csvs(kt_dir, "_kernel_stats.csv"):
        stats += list(csv.DictReader(open(f)))
    tile = [r for r in stats if r["Name"].startswith(prefix)]
    if len(tile) != 1:
        raise SystemExit("expected one tile-kernel row in the kernel stats, found %d" % len(tile))
    tile = tile[0]
    durs = []
    for f in _csvs(kt_dir, "_kernel_trace.csv"):
        for r in csv.DictReader(open(f)):
            if r["Kernel_Name"].startswith(prefix):
                durs.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    durs = [d for _, d in sorted(durs)][warmup:]
    steady_ns = sum(durs) / max(len(durs), 1)
    per = _counter_means(pmc_dirs)
    tiles = [k for k in per if k.startswith(prefix)]
    if len(tiles) != 1:
        raise SystemExit("expected one tile kernel in the counter runs, found %s" % tiles)
    tk = per[tiles[0]]
    shapes = {(v[1], v[2] // v[1]) for vals in tk.values() for v in vals}
    if len(shapes) != 1:
        raise SystemExit("tile kernel launched with several shapes: %s" % sorted(shapes))
    (block, grid), = shapes

    def mean(kern, name):
        vals = per.get(kern, {}).get(name)
        return None if not vals else sum(v[0] for v in vals) / len(vals)

    def calib(pred, name):
        vals = [max(v[0] for v in c[name]) for k, c in per.items() if pred(k) and name in c]
        return max(vals) if vals else None

    kib = COPY_BYTES / 1024.0
    gather_read_kib = kib + (COPY_BYTES // 64) * 8 / 1024.0
    def is_gather(k):
        kl = k.lower()
        return ("index" in kl or "gather" in kl) and not any(w in kl for w in ("sort", "radix", "randperm", "arange",
                                                                             "scan", "fill", "reduce"))

    sum_fetch = calib(lambda k: "reduce_kernel" in k, "FETCH_SIZE")
    gather_fetch = calib(is_gather, "FETCH_SIZE")
    fill_write = calib(lambda k: "FillFunctor<float>" in k, "WRITE_SIZE")
    big = sorted(((max(v[0] for v in c["FETCH_SIZE"]), k) for k, c in per.items()
                  if "FETCH_SIZE" in c and not k.startswith(TILE_PREFIX)), reverse=True)[:4]
    lines = ["# rocprofv3 summary: tile kernel k_tiles<lin, fp32c> (linearize, compensated FP32), %s" % workload,
             "#", "# commands (from /tmp, TMPDIR=/tmp, REPO = the repository root):"]
    lines += ["#   " + c for c in command] + ["#"]
    lines += ["# largest FETCH_SIZE (KiB) of other kernels: " + "; ".join("%.0f %s" % (v, k[:80]) for v, k in big)]
    lines += ["kernel: %s" % tile["Name"].split("(")[0],
              "launch: block %d tile %d grid %d order %d" % (block, tile_points, grid, tile_order),
              "kernel_sources_sha256: %s" % kernel_sources_sha256(),
              "tile_kernel_calls: %s" % tile["Calls"],
              "tile_kernel_avg_ns: %.0f" % float(tile["AverageNs"]),
              "tile_kernel_min_ns: %s" % tile["MinNs"],
              "tile_kernel_max_ns: %s" % tile["MaxNs"],
              "tile_kernel_steady_avg_ns: %.0f (%d dispatches after %d warm-up steps)" % (steady_ns, len(durs), warmup)]
    for name in sorted(tk):
        lines.append("counter %s: %.6e (mean of %d dispatches)" % (name, mean(tiles[0], name), len(tk[name])))
    fetch = mean(tiles[0], "FETCH_SIZE")
    write = mean(tiles[0], "WRITE_SIZE")
    if sum_fetch and fill_write and fetch is not None and write is not None:
        s_stream = kib / sum_fetch
        s_gather = gather_read_kib / gather_fetch if gather_fetch else None
        w_scale = kib / fill_write
        lines += ["calibration_sum_fetch_kib: %.1f (streams %.1f KiB: 128-byte requests counted as 64)" % (
                      sum_fetch, kib),
                  "calibration_gather_fetch_kib: %s (%.1f KiB of 64-byte rows + indices: each row's miss moves a "
                  "128-byte line)" % ("%.1f" % gather_fetch if gather_fetch else "n/a", gather_read_kib),
                  "calibration_fill_write_kib: %.1f (writes %.1f KiB)" % (fill_write, kib),
                  "fetch_scale_stream: %.4f" % s_stream,
                  "fetch_scale_gather: %s" % ("%.4f" % s_gather if s_gather else "n/a"),
                  "write_scale: %.4f" % w_scale]
        lo = fetch * 1024.0 + write * w_scale * 1024.0
        hi = fetch * s_stream * 1024.0 + write * w_scale * 1024.0
        lines += ["traffic_bytes_per_launch_range: %.6e %.6e (read requests all 64 B / all 128 B)" % (lo, hi)]
        rd = mean(tiles[0], "TCC_EA0_RDREQ_sum")
        r32 = mean(tiles[0], "TCC_EA0_RDREQ_32B_sum")
        r128 = mean(tiles[0], "TCC_BUBBLE_sum")
        if rd is not None and r32 is not None and r128 is not None and r128 > 0.01 * rd:
            exact = 128.0 * r128 + 64.0 * (rd - r128 - r32) + 32.0 * r32 + write * w_scale * 1024.0
            lines.append("traffic_bytes_per_launch: %.6e (read requests by size: 128 B %.4g, 32 B %.4g, 64 B the rest)"
                         % (exact, r128, r32))
        else:
            lines.append("traffic_bytes_per_launch: %.6e (midpoint of the range: the 128-byte request counter "
                         "reads %s here, so the split of requests by size is unknown)" % (
                             (lo + hi) / 2, "n/a" if r128 is None else "%.3g" % r128))
    hit, miss = mean(tiles[0], "TCC_HIT_sum"), mean(tiles[0], "TCC_MISS_sum")
    if hit is not None and miss is not None and hit + miss > 0:
        lines.append("l2_hit_rate: %.4f" % (hit / (hit + miss)))
    valu = mean(tiles[0], "SQ_INSTS_VALU")
    if valu is not None:
        lines.append("valu_insts_per_dispatch: %.6e" % valu)
        lines.append("valu_issue_frac_at_steady_time: %.4f (x 4 cycles / (1024 SIMDs x %.0f ns x 2.4 GHz))" % (
            valu * 4 / (SIMDS * steady_ns * 1e-9 * CLOCK_HZ), steady_ns))
        gui = mean(tiles[0], "GRBM_GUI_ACTIVE")
        if gui:
            lines.append("valu_issue_frac_at_busy_cycles: %.4f (x 4 cycles / (128 SIMDs per XCD x GRBM_GUI_ACTIVE "
                         "%.4g, read as busy cycles summed over the 8 XCDs: %.3g GHz over the steady time)" % (
                             valu * 4 / (SIMDS / 8 * gui), gui, gui / 8 / (steady_ns * 1e-9) / 1e9))
    lines += ["", "top kernels of the kernel-trace run (total time):", "| calls | avg us | total ms | % | kernel |",
              "|---|---|---|---|---|"]
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in stats[:10]:
        lines.append("| %s | %.1f | %.2f | %.1f | %s |" % (r["Calls"], float(r["AverageNs"]) / 1e3,
                                                       float(r["TotalDurationNs"]) / 1e6,
                                                       float(r["Percentage"]), r["Name"][:110]))
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
    out = torch.empty((batch.F, 43), dtype=torch.float64, device="cuda")
    inl_d = torch.empty((batch.F, batch.L), dtype=torch.int64, device="cuda")
    for _ in range(warmup):
        batch.linearize_async(d_poses, out, inl_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.linearize_async(d_poses, out, inl_d)
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
    tk = batch.time_kernels(poses, reps=20)
    walked, chunks, lookups = batch.work()
    B_walk = work_bytes(walked.sum(), lookups.sum(), hits, len(pairs))
    B_every = work_bytes(pts, pts * L, hits, len(pairs))
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
           "roofline": make_roofline(B_walk, B_every, None, tk, None, "k_tiles<lin,%s>" % args.precision)}
    print(json.dumps(out), flush=True)
    batch.close()
    for x in srcs + maps + clouds:
        x.close()
    ctx.close()


def _oracle_threads(fn, items, cores):
    with ThreadPoolExecutor(cores) as ex:
        return list(ex.map(fn, items))


def bench_diff(args):
    """Differentiation batch: 64 factors x 100k source points (config-1 scenes,
    0.5 m voxels).  A step is, for every factor, the forward error and the
    backward kernel: de/dxi (6 per factor) and de/dmu (FP32, 6.4M x 3), all on
    device pointers.  Accuracy: sampled factors against the FP64 oracle's exact
    gradient on the device's correspondences."""
    import torch
    import oracle
    import synth
    from oracle.parity import frozen_from_device_keys, rel_err
    from paper_2407_10344_amd import vgicp
    t = time.time()
    cfg = synth.config4()
    log("generated differentiation batch in %.1f s" % (time.time() - t))
    ctx = vgicp.Context(0)
    maps, srcs, batch = vgicp.build_workload(ctx, cfg, precision=args.precision, use_graph=True)
    F = len(cfg["factors"])
    poses = np.array(cfg["poses"])
    n_src = np.array([cfg["sources"][s].n for (s, _) in cfg["factors"]])
    pts = int(n_src.sum())
    d_T = torch.tensor(vgicp.poses12(poses), device="cuda")
    ge = torch.ones(F, dtype=torch.float64, device="cuda")

    def step():
        e = batch.evaluate_async(d_T)
        gxi, gp = batch.backward_async(d_T, ge, points_dtype=torch.float32)
        return e, gxi, gp

    def timed(fn, k):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k, r

    dt, (e, gxi, gp) = timed(step, args.steps)
    dt_fwd, _ = timed(lambda: batch.evaluate_async(d_T), args.steps)
    dt_bwd, _ = timed(lambda: batch.backward_async(d_T, ge, points_dtype=torch.float32), args.steps)
    log("fwd+bwd %.3f ms/step (fwd %.3f, bwd %.3f)" % (dt * 1e3, dt_fwd * 1e3, dt_bwd * 1e3))
    e, gxi, gp = e.cpu().numpy(), gxi.cpu().numpy(), gp.cpu().numpy()
    # accuracy on sampled factors
    omaps = {}
    worst = {"e": 0.0, "grad_xi": 0.0, "grad_points": 0.0}
    for f in (0, 21, 42, 63):
        s, tg = cfg["factors"][f]
        of = oracle.factor_from_clouds(cfg["sources"][s], cfg["targets"][tg], cfg["resolutions"])
        kd, fd = batch.correspondences(poses[f], f)
        fz, _ = frozen_from_device_keys(of, poses[f], kd, fd)
        g_o, gm_o = of.gradient(poses[f], frozen=fz)
        row0, n = batch.source_rows[id(srcs[s])]
        worst["e"] = max(worst["e"], rel_err(e[f], of.evaluate(poses[f], frozen=fz)))
        worst["grad_xi"] = max(worst["grad_xi"], rel_err(gxi[f], g_o))
        worst["grad_points"] = max(worst["grad_points"], rel_err(gp[row0:row0 + n].astype(np.float64), gm_o))
    log("worst relative errors on 4 sampled factors: %s" % worst)
    cpu = None
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        ofs = _oracle_threads(lambda f: oracle.factor_from_clouds(cfg["sources"][cfg["factors"][f][0]],
                                                                  cfg["targets"][cfg["factors"][f][1]],
                                                                  cfg["resolutions"]), range(F), cores)
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            _oracle_threads(lambda f: (ofs[f].evaluate(poses[f]), ofs[f].gradient(poses[f])), range(F), cores)
            times.append(time.perf_counter() - t0)
        cpu = {"value": pts / float(np.median(times)), "unit": "source points/s (forward + backward)",
               "cores": cores, "kind": "oracle", "cpu": cpu_model(), "runs": 5,
               "sample": "all %d factors (%d source points): FP64 oracle evaluate + exact gradient, one factor "
                         "per thread, median of 5 runs of %.2f-%.2f s" % (F, pts, min(times), max(times))}
        log("cpu baseline", cpu)
    out = {"metric": "source points differentiated/sec (forward e + backward de/dxi, de/dmu)",
           "value": pts / dt, "unit": "source points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp32c": "f32", "fp32": "f32", "fp64": "f64"}[args.precision], "data": "synthetic",
           "config": {"workload": "differentiation batch", "factors": F, "source_points_per_factor": 100_000,
                      "voxel_m": 0.5, "levels": 1, "precision": args.precision, "total_source_points": pts,
                      "point_gradient_dtype": "float32", "pose": "configured linearization point (initial guess)"},
           "parts_ms": {"forward": dt_fwd * 1e3, "backward": dt_bwd * 1e3},
           "accuracy_vs_oracle": dict(worst, factors=[0, 21, 42, 63],
                                      note="oracle exact gradient on the device's correspondences"),
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    batch.close()
    ctx.close()


def _pose_error(Ta, Tb):
    """Rotation angle (deg) and translation (m) of Ta^-1 Tb; the angle from
    atan2(|sin|, cos) so that tiny rotations do not round to zero."""
    D = np.linalg.inv(Ta) @ Tb
    Rm = D[:3, :3]
    s = 0.5 * np.linalg.norm([Rm[2, 1] - Rm[1, 2], Rm[0, 2] - Rm[2, 0], Rm[1, 0] - Rm[0, 1]])
    c = (np.trace(Rm) - 1) / 2
    return math.degrees(math.atan2(s, c)), float(np.linalg.norm(D[:3, 3]))


def bench_precision(args):
    """Precision stress: 4 factors of 1M source points 10 km from the origin.  Each
    precision mode drives a 10-iteration Levenberg-Marquardt loop (device
    resident, FP64 6x6 solves); the final poses are compared with the FP64
    oracle's LM on the same inputs, and e/H/b at the first linearization with the
    oracle's.  A step is one 10-iteration LM run of the batch."""
    import torch
    import oracle
    import synth
    from oracle.parity import ASSERTED, block_errors, expected_with_device_keys, rel_err
    from paper_2407_10344_amd import vgicp
    t = time.time()
    cfg = synth.config5()
    log("generated precision-stress batch in %.1f s" % (time.time() - t))
    F = len(cfg["factors"])
    poses = np.array(cfg["poses"])
    n_src = np.array([cfg["sources"][s].n for (s, _) in cfg["factors"]])
    pts = int(n_src.sum())
    iters = 10
    cores = len(os.sched_getaffinity(0))
    ofs = _oracle_threads(lambda f: oracle.factor_from_clouds(cfg["sources"][f], cfg["targets"][f],
                                                              cfg["resolutions"]), range(F), cores)
    t0 = time.perf_counter()
    refs = _oracle_threads(lambda f: ofs[f].lm(poses[f], iters=iters, lambda0=1e-4), range(F), cores)
    t_oracle = time.perf_counter() - t0
    ctx = vgicp.Context(0)
    modes = {}
    for prec in ("fp32", "fp32c", "fp64"):
        maps, srcs, batch = vgicp.build_workload(ctx, cfg, precision=prec, use_graph=True)
        for _ in range(max(1, args.warmup)):
            T, acc, eh = batch.lm(poses, iters=iters, lambda0=1e-4)
        torch.cuda.synchronize()
        k = max(1, min(args.steps, 10))
        t0 = time.perf_counter()
        for _ in range(k):
            T, acc, eh = batch.lm(poses, iters=iters, lambda0=1e-4)
        dt = (time.perf_counter() - t0) / k
        errs = [_pose_error(refs[f]["pose"], T[f]) for f in range(F)]
        same_acc = [bool(np.array_equal(acc[f], refs[f]["accepted"])) for f in range(F)]
        e0, H0, b0, _ = batch.linearize(poses)
        lin = {}
        for f in range(F):
            if prec == "fp32":
                r = ofs[f].linearize(poses[f])
                d = {"e": rel_err(e0[f], r["e"]), "H": rel_err(H0[f], r["H"]), "b": rel_err(b0[f], r["b"])}
            else:
                kd, fd = batch.correspondences(poses[f], f)
                ee, HH, bb, _ = expected_with_device_keys(ofs[f], poses[f], kd, fd)
                d = {"e": rel_err(e0[f], ee), "H": rel_err(H0[f], HH), "b": rel_err(b0[f], bb)}
                d.update(block_errors(H0[f], b0[f], HH, bb, ofs[f].gradient_scale(poses[f])))
                d = {kk: d[kk] for kk in ASSERTED}
            lin = {kk: max(lin.get(kk, 0.0), v) for kk, v in d.items()}
        modes[prec] = {"lm_ms": dt * 1e3, "point_evaluations_per_s": pts * 2 * iters / dt,
                       "final_rotation_error_deg_max": max(x[0] for x in errs),
                       "final_translation_error_m_max": max(x[1] for x in errs),
                       "accept_sequence_equal_to_oracle": same_acc,
                       "iteration0_rel_err_max": lin}
        log(prec, modes[prec])
        batch.close()
        for x in list(maps.values()) + list(srcs.values()):
            x.close()
    r0 = [_pose_error(cfg["poses_true"][f], refs[f]["pose"]) for f in range(F)]
    cpu = {"value": pts * 2 * iters / t_oracle, "unit": "source point evaluations/s", "cores": min(cores, F),
           "kind": "oracle", "cpu": cpu_model(),
           "sample": "the whole workload: the FP64 oracle's %d-iteration LM of the %d factors, one factor per thread "
                     "(%.2f s)" % (iters, F, t_oracle)}
    m = modes["fp32c"]
    out = {"metric": "source point evaluations/sec in a 10-iteration Levenberg-Marquardt loop "
                     "(linearize + evaluate per iteration), with the final pose error against the FP64 oracle",
           "value": m["point_evaluations_per_s"], "unit": "source point evaluations/s", "n_gpus": 1,
           "steps": max(1, min(args.steps, 10)), "warmup": max(1, args.warmup), "ms_per_step": m["lm_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "precision stress", "factors": F, "source_points_per_factor": int(n_src[0]),
                      "target_points_per_factor": int(cfg["targets"][0].n), "offset_from_origin_km": 10,
                      "voxel_m": cfg["resolutions"], "lm_iterations": iters, "lambda0": 1e-4,
                      "value_mode": "fp32c (compensated FP32)"},
           "modes": modes,
           "oracle_lm_vs_truth": {"rotation_deg_max": max(x[0] for x in r0),
                                  "translation_m_max": max(x[1] for x in r0)},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="global",
                    choices=["global", "odometry", "single", "preprocess", "local", "diff", "precision"])
    ap.add_argument("--submaps", type=int, default=500)
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp32", "fp64"])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-tune-cache", action="store_true", help="autotune from scratch (ignore the tuned shapes)")
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0: library default / tuned)")
    ap.add_argument("--tile", type=int, default=0, help="source points per tile (0: default / tuned)")
    ap.add_argument("--bpc", type=int, default=0, help="persistent workgroups per CU (0: default / tuned)")
    ap.add_argument("--tile-order", type=int, default=0,
                    help="1: contiguous tile range per XCD, 2: tiles dealt round-robin to XCDs (0: default / tuned)")
    ap.add_argument("--lane-kahan", action="store_true", help="Kahan-compensated FP32 sums inside each lane")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run --warmup + this many batched steps (for profilers), print no JSON")
    ap.add_argument("--summarize-profiles", nargs="+", metavar="DIR",
                    help="write the text summary of rocprofv3 runs of --profile-steps (a kernel-trace run, "
                         "then counter runs) and exit")
    ap.add_argument("--workload-cache", default=None,
                    help="npz file holding the generated global batch: written on the first run, read after "
                         "(saves regenerating it for every profiler pass)")
    ap.add_argument("--profile-command", action="append", default=[],
                    help="command line recorded in the summary (repeatable)")
    args = ap.parse_args()
    if args.summarize_profiles:
        tag = "global submap batch, %d submaps" % args.submaps if args.workload == "global" else args.workload
        sys.stdout.write(summarize_profiles(args.summarize_profiles[0], args.summarize_profiles[1:],
                                            args.profile_command, args.tile, args.tile_order or 1, tag, args.warmup,
                                            args.block))
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
    if args.workload == "diff":
        bench_diff(args)
        return
    if args.workload == "precision":
        bench_precision(args)
        return
    cfg, desc = make_workload(args.workload, args.submaps, args.workload_cache)
    ctx = vgicp.Context(0)
    t = time.time()
    shape = {"block": args.block, "tile": args.tile, "blocks_per_cu": args.bpc, "tile_order": args.tile_order}
    tune_cache = None if any(shape.values()) or args.no_tune_cache else TUNE_CACHE
    maps, srcs, batch = vgicp.build_workload(ctx, cfg, precision=args.precision, use_graph=True,
                                             lane_kahan=args.lane_kahan, tune_cache=tune_cache, **shape)
    torch.cuda.synchronize()
    log("device maps/sources/batch built in %.1f s" % (time.time() - t))
    poses = vgicp.poses12(np.array(cfg["poses"]))
    info = batch.info()
    if not args.no_tune and not any(shape.values()):
        t = time.time()
        chosen = batch.tune(poses, reps=2)
        info = batch.info()
        log("autotuned %s in %.1f s" % (chosen, time.time() - t))

    if args.profile_steps:
        # the steps as the bench times them: device-resident poses and results,
        # launched back to back, one synchronization at the end
        d_poses = torch.tensor(np.ascontiguousarray(poses), dtype=torch.float64, device="cuda")
        out = torch.empty((batch.F, 43), dtype=torch.float64, device="cuda")
        inl_d = torch.empty((batch.F, batch.L), dtype=torch.int64, device="cuda")
        for _ in range(args.warmup + args.profile_steps):
            batch.linearize_async(d_poses, out, inl_d)
        torch.cuda.synchronize()
        # kernels of known traffic, to scale the memory counters: a fill that
        # writes COPY_BYTES, a reduction that streams them, and a gather of
        # 64-byte rows in random order (the size of the kernel's record gathers)
        src_t = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        total = src_t.sum()
        rows = src_t.view(-1, 16)
        perm = torch.randperm(rows.shape[0], device="cuda")
        torch.cuda.synchronize()
        gathered = torch.index_select(rows, 0, perm)
        torch.cuda.synchronize()
        log("profile run done: %d + %d warm-up linearize steps; calibration: fill (write), sum (read) and "
            "64-byte row gather of %d bytes, %s %s" % (args.profile_steps, args.warmup, COPY_BYTES, float(total),
                                                      tuple(gathered.shape)))
        return

    dt, dt_host, (e, H, b, inl), same = time_steps(batch, poses, args.steps, args.warmup)
    log("device-resident %.3f ms/step, host buffers %.3f ms/step, identical results: %s"
        % (dt * 1e3, dt_host * 1e3, same))
    n_src = np.array([cfg["sources"][s].n for (s, _) in cfg["factors"]], dtype=np.int64)
    pts = int(n_src.sum())
    hits = int(inl.sum())
    value = pts / dt

    # dominant kernel time, HIP events on the library's stream; the work counts of
    # its last launch (the same every launch: same poses, same culling)
    tk = batch.time_kernels(poses, reps=max(3, min(args.steps, 20)))
    walked, chunks, lookups = batch.work()
    work = {"walked_points": int(walked.sum()), "walked_chunks": int(chunks.sum()), "lookups": int(lookups.sum()),
            "hits": hits, "culled_point_fraction": 1.0 - walked.sum() / max(pts, 1)}
    B_walk = work_bytes(walked.sum(), lookups.sum(), hits, len(n_src))
    B_every = work_bytes(pts, pts * inl.shape[1], hits, len(n_src))
    footprint = unique_footprint(cfg, maps)
    overlap = inl[:, 0] / np.maximum(n_src, 1)
    overlap_desc = {"percentiles_5_25_50_75_95": np.percentile(overlap, [5, 25, 50, 75, 95]).round(4).tolist(),
                    "fraction_in_0.1_0.6": float(np.mean((overlap >= 0.1) & (overlap <= 0.6))),
                    "definition": "fraction of a factor's source points in an occupied target voxel"}

    # plain per-factor path (one upload, launch, download and sync per factor): with the
    # batch's launch shape, and with its own tuned shape (small tiles fill the device
    # from one factor)
    plain = None
    if args.plain_steps > 0:
        plain = {}
        for name, kw in (("batch_shape", dict(block=info["block_threads"], tile=info["tile_points"],
                                              tile_order=info["tile_order"])), ("tuned", {})):
            _, _, pb = vgicp.build_workload(ctx, cfg, precision=args.precision, use_graph=False, plain=True, **kw)
            if name == "tuned":
                chosen = pb.tune(poses, reps=1)
                log("plain path tuned: %s" % chosen)
            pb.linearize(poses)
            t0 = time.perf_counter()
            for _ in range(args.plain_steps):
                ep, Hp, bp, _ = pb.linearize(poses)
            plain_dt = (time.perf_counter() - t0) / args.plain_steps
            pi = pb.info()
            plain[name] = {"value": pts / plain_dt, "ms_per_step": plain_dt * 1e3,
                           "batched_speedup": plain_dt / dt_host,
                           "launch": {"block_threads": pi["block_threads"], "tile_points": pi["tile_points"]}}
            if name == "batch_shape":
                plain[name]["bitwise_equal_to_batched"] = bool(
                    np.array_equal(ep, e) and np.array_equal(Hp, H) and np.array_equal(bp, b))
            pb.close()
            log("plain per-factor (%s): %.1f ms/step" % (name, plain_dt * 1e3))
        plain["unit"] = "source points/s"
        plain["speedup_basis"] = "plain loop vs the batched host-buffer call (both upload poses and download results)"

    prof_path = profile_summary_path(args.workload, args.submaps, args.precision)
    counters = measured_counters(prof_path, info)
    log("profile counters: %s (%s)" % (counters, os.path.relpath(prof_path, ROOT)))
    roofline = make_roofline(B_walk, B_every, footprint, tk, counters, "k_tiles<lin,%s>" % args.precision)

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
                       hit_rate=hits / max(pts, 1), launch=info, overlap_rate=overlap_desc, work=work),
        "host_buffers": {"value": pts / dt_host, "ms_per_step": dt_host * 1e3,
                         "includes": "pose upload and result download"},
        "plain": plain,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_sample": parity,
    }
    print(json.dumps(out), flush=True)
    batch.close()


def work_bytes(points, lookups, hits, factors):
    """Algorithmic bytes of a launch: 36 B per source point read, 8 B per table
    lookup, 36 B per voxel hit, 392 B per factor (pose in, result out)."""
    return int(points) * B_POINT + int(lookups) * B_KEY + int(hits) * B_HIT + int(factors) * B_FACTOR


def unique_footprint(cfg, maps):
    """Bytes one launch must touch at least once: every distinct source's points and
    covariances (36 B per point) and every distinct target map's voxel records
    (64 B) and block-table entries (16 B)."""
    srcs = sorted({s for (s, _) in cfg["factors"]})
    b = sum(cfg["sources"][s].n for s in srcs) * B_POINT
    for m in maps.values():
        for l in range(m.L):
            V, cap = m.info(l)
            b += V * 64 + cap * 16
    return int(b)


def make_roofline(B_walk, B_every, footprint, tk, counters, kernel):
    """The roofline object of the bench line: HBM fraction of the algorithmic bytes
    of the walked work, the DRAM fraction and VALU issue fraction from the counters.
    `bound` is the higher of the VALU fraction and the HBM-side fraction, which is
    the DRAM fraction the counters measured when there is one (the walked-work
    bytes include sources that the factors sharing them read from L2 and the
    last-level cache, and can exceed what HBM delivers), else the walked one."""
    t = tk["tile_kernel_ms"] * 1e-3
    hbm = B_walk / t / HBM_PEAK
    valu = None
    if counters and counters.get("valu_insts") is not None:
        valu = counters["valu_insts"] * 64 / t / VALU_PEAK
    traffic = counters.get("traffic_bytes") if counters else None
    r = {"kernel": kernel, "kernel_ms": tk["tile_kernel_ms"], "reduce_ms": tk["reduce_ms"],
         "algorithmic_bytes": int(B_walk), "algorithmic_bytes_every_point": int(B_every),
         "hbm_frac": hbm, "hbm_frac_every_point": B_every / t / HBM_PEAK,
         "unique_footprint_bytes": footprint, "traffic": traffic,
         "dram_frac": None if traffic is None else traffic / t / HBM_PEAK,
         "l2_hit_rate": counters.get("l2_hit_rate") if counters else None,
         "valu_issue_frac": valu,
         "counters_from": counters.get("source") if counters else None}
    dram = r["dram_frac"]
    hbm_side = dram if dram is not None else hbm
    if valu is not None and valu > hbm_side:
        r.update({"bound": "alu", "achieved": counters["valu_insts"] * 64 / t / 1e12, "peak": VALU_PEAK / 1e12,
                  "unit": "TOP/s", "frac": valu,
                  "achieved_is": "VALU lane operations/s (wave64 VALU instructions from the counters x 64 / "
                                 "kernel time); peak = 1024 SIMDs x 16 lanes x 2.4 GHz"})
    else:
        r.update({"bound": "hbm", "achieved": B_walk / t / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                  "frac": hbm,
                  "achieved_is": "algorithmic bytes of the walked work / kernel time: 36 B per walked source "
                                 "point, 8 B per table lookup, 36 B per voxel hit, 392 B per factor"})
    return r


if __name__ == "__main__":
    main()
