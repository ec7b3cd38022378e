"""Seeded workload builders.

Five workloads mirror the factor batches the method linearizes (Sec. III-C,
IV-B, V-B): a single scan-to-scan factor, an odometry batch against keyframes,
a global submap-to-submap batch, a differentiation batch and a precision
stress batch.  Every builder is deterministic in its seed
(``numpy.random.SeedSequence``) and returns plain numpy data.

Pose convention: a factor's pose T = (R, t) maps source-frame points into the
target frame, y = R mu + t.  Poses are 4x4 float64 arrays here and 12 doubles
(R row-major, then t) at the library/oracle boundary.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

from .clouds import Cloud, make_cloud
from .scene import random_boxes, raycast, sample_surfaces


# ----------------------------------------------------------------------------
# small pose helpers (input construction only)


def _rng(*entropy):
    return np.random.default_rng(np.random.SeedSequence([int(e) for e in entropy]))


def pose_from(Rm, t):
    T = np.eye(4)
    T[:3, :3] = Rm
    T[:3, 3] = t
    return T


def inv_pose(T):
    Ti = np.eye(4)
    Ti[:3, :3] = T[:3, :3].T
    Ti[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return Ti


def apply_pose(T, x):
    return x @ T[:3, :3].T + T[:3, 3][None, :]


def unit_vector(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def random_pose(rng, angle_deg, trans_m):
    """Rotation of exactly ``angle_deg`` about a uniform axis, translation of ``trans_m``."""
    Rm = Rotation.from_rotvec(unit_vector(rng) * math.radians(angle_deg)).as_matrix()
    return pose_from(Rm, unit_vector(rng) * trans_m)


def pose12(T):
    return np.concatenate([T[:3, :3].reshape(-1), T[:3, 3]]).astype(np.float64)


def yaw_pose(x, y, z, yaw):
    return pose_from(Rotation.from_euler("z", yaw).as_matrix(), np.array([x, y, z]))


# ----------------------------------------------------------------------------
# config 1 / 4 / 5: the single-factor scene


def _scene1(rng):
    return random_boxes(rng, 20, (-18.0, -18.0), (18.0, 18.0), 1.0, 5.0)


def config1(seed=1, n_target=20000, n_source=5000, resolutions=(0.5,), translate_km=0.0,
            angle_deg=5.0, trans_m=0.3, workers=-1):
    """Ground plane over [-20, 20]^2 plus 20 boxes (sides 1-5 m), sigma = 0.02 m.

    Target and source are independent area-uniform draws of the same scene;
    the source is expressed in a frame offset by a (5 deg, 0.3 m) pose, so the
    true source->target pose is ``pose_true`` and the factor is linearized at
    ``pose_init`` = identity.  With ``translate_km`` > 0 the whole scene is
    shifted by that distance along a seeded horizontal direction and the
    offset rotation is applied about the source centroid.
    """
    seed = seed if isinstance(seed, (tuple, list)) else (seed,)
    scene_rng, samp_rng, pose_rng, shift_rng = (np.random.default_rng(s) for s in
                                                np.random.SeedSequence(list(seed)).spawn(4))
    lo, hi = _scene1(scene_rng)
    tgt = sample_surfaces(samp_rng, lo, hi, (-20.0, -20.0), (20.0, 20.0), n_target)
    srcw = sample_surfaces(samp_rng, lo, hi, (-20.0, -20.0), (20.0, 20.0), n_source)
    sensor = np.array([0.0, 0.0, 1.8])
    T_off = random_pose(pose_rng, angle_deg, trans_m)
    if translate_km > 0:
        phi = shift_rng.uniform(0, 2 * math.pi)
        D = 1000.0 * translate_km * np.array([math.cos(phi), math.sin(phi), 0.0])
        tgt = tgt + D
        srcw = srcw + D
        sensor = sensor + D
        c = srcw.mean(axis=0)
        Rm = T_off[:3, :3]
        T_off = pose_from(Rm, c - Rm @ c + T_off[:3, 3])
    src = apply_pose(inv_pose(T_off), srcw)
    vp_src = apply_pose(inv_pose(T_off), sensor[None])[0]
    snap = max(resolutions)
    target = make_cloud(tgt, sensor, snap, workers=workers)
    source = make_cloud(src, vp_src, snap, workers=workers)
    return {
        "name": "single factor",
        "targets": [target],
        "sources": [source],
        "resolutions": list(resolutions),
        "factors": [(0, 0)],
        "poses": [np.eye(4)],
        "poses_true": [T_off],
        "target_viewpoints": [sensor],
    }


def _config4_instance(j, n_points, workers):
    return config1(seed=(4, j), n_target=n_points, n_source=n_points, workers=workers)


def config4(n_factors=64, n_points=100_000, processes=None):
    """64 independent config-1 instances with 100k source and 100k target points."""
    procs = processes or min(16, os.cpu_count() or 1, n_factors)
    if procs > 1:
        with ProcessPoolExecutor(procs) as ex:
            inst = list(ex.map(_config4_instance, range(n_factors), [n_points] * n_factors,
                               [1] * n_factors))
    else:
        inst = [_config4_instance(j, n_points, -1) for j in range(n_factors)]
    return _stack_instances(inst, "differentiation")


def _config5_instance(j, n_points, workers):
    return config1(seed=(5, j), n_target=n_points, n_source=n_points, translate_km=10.0,
                   workers=workers)


def config5(n_factors=4, n_points=1_000_000, processes=None):
    """4 config-1 instances with 1M + 1M points, shifted 10 km from the origin."""
    procs = processes or min(4, os.cpu_count() or 1, n_factors)
    w = max(1, (os.cpu_count() or 1) // procs)
    if procs > 1:
        with ProcessPoolExecutor(procs) as ex:
            inst = list(ex.map(_config5_instance, range(n_factors), [n_points] * n_factors,
                               [w] * n_factors))
    else:
        inst = [_config5_instance(j, n_points, -1) for j in range(n_factors)]
    return _stack_instances(inst, "precision stress")


def _stack_instances(inst, name):
    out = {"name": name, "targets": [], "sources": [], "resolutions": inst[0]["resolutions"],
           "factors": [], "poses": [], "poses_true": [], "target_viewpoints": []}
    for j, d in enumerate(inst):
        out["targets"].append(d["targets"][0])
        out["sources"].append(d["sources"][0])
        out["factors"].append((j, j))
        out["poses"].append(d["poses"][0])
        out["poses_true"].append(d["poses_true"][0])
        out["target_viewpoints"].append(d["target_viewpoints"][0])
    return out


# ----------------------------------------------------------------------------
# config 2: odometry batch from a simulated spinning LiDAR


def _smooth_trajectory(rng, length, step=0.05):
    """Smooth random planar path: heading is a sum of low-frequency sinusoids."""
    s = np.arange(0.0, length + step, step)
    yaw0 = rng.uniform(0, 2 * math.pi)
    amp = rng.uniform(0.05, 0.25, 3)
    freq = rng.uniform(0.02, 0.08, 3)
    ph = rng.uniform(0, 2 * math.pi, 3)
    yaw = yaw0 + sum(a * np.sin(2 * math.pi * f * s + p) for a, f, p in zip(amp, freq, ph))
    x = np.concatenate([[0.0], np.cumsum(np.cos(yaw[:-1]) * step)])
    y = np.concatenate([[0.0], np.cumsum(np.sin(yaw[:-1]) * step)])
    x -= x[-1] / 2
    y -= y[-1] / 2
    return s, x, y, yaw


def _lidar_dirs(n_rings=32, n_az=1000, elev=(-15.0, 15.0)):
    el = np.radians(np.linspace(elev[0], elev[1], n_rings))
    az = np.linspace(0, 2 * math.pi, n_az, endpoint=False)
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1).reshape(-1, 3)


def lidar_frame(rng, T_sensor, lo, hi, dirs, rmin=1.0, rmax=80.0, noise=0.02):
    """Points (sensor frame) returned by one sweep of the spinning LiDAR at pose T_sensor."""
    dw = dirs @ T_sensor[:3, :3].T
    t = raycast(T_sensor[:3, 3], dw, lo, hi)
    ok = np.isfinite(t) & (t >= rmin) & (t <= rmax)
    pts = dirs[ok] * t[ok, None]
    return pts + rng.normal(0.0, noise, pts.shape)


def _urban_scene(scene_rng, path):
    """Ground + 200 boxes (footprint 2-15 m, height 2-25 m) in [-75, 75]^2 m, kept
    3 m clear of the trajectory, and 40 m perimeter walls so most rays return."""
    tree = cKDTree(path)
    boxes_lo, boxes_hi = [], []
    while len(boxes_lo) < 200:
        lo, hi = random_boxes(scene_rng, 64, (-75.0, -75.0), (75.0, 75.0), 2.0, 15.0, 2.0, 25.0)
        for b in range(lo.shape[0]):
            c = (lo[b, :2] + hi[b, :2]) / 2
            half = (hi[b, :2] - lo[b, :2]) / 2
            # clearance: no trajectory sample within 3 m of the footprint
            near = tree.query_ball_point(c, float(np.linalg.norm(half)) + 3.0)
            if near:
                d = np.maximum(np.abs(path[near] - c) - half, 0.0)
                if np.min(np.linalg.norm(d, axis=1)) < 3.0:
                    continue
            boxes_lo.append(lo[b])
            boxes_hi.append(hi[b])
            if len(boxes_lo) == 200:
                break
    lo = np.array(boxes_lo)
    hi = np.array(boxes_hi)
    W, th, H = 70.0, 1.0, 40.0
    walls_lo = np.array([[-W - th, -W - th, 0], [W, -W - th, 0], [-W - th, -W - th, 0], [-W - th, W, 0]])
    walls_hi = np.array([[-W, W + th, H], [W + th, W + th, H], [W + th, -W, H], [W + th, W + th, H]])
    return np.concatenate([lo, walls_lo]), np.concatenate([hi, walls_hi])


def raw_frame(seed=6, n_rings=128, n_az=1024, elev=(-45.0, 45.0)):
    """One raw sweep of a 128-ring, 90-degree-FOV spinning LiDAR in the urban block
    (the preprocessing input): points in the sensor frame, sensor at the origin."""
    scene_rng, traj_rng, noise_rng = (np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(3))
    s, x, y, yaw = _smooth_trajectory(traj_rng, 20.0)
    lo, hi = _urban_scene(scene_rng, np.stack([x, y], axis=1))
    i = len(s) // 2
    pts = lidar_frame(noise_rng, yaw_pose(x[i], y[i], 1.8, yaw[i]), lo, hi, _lidar_dirs(n_rings, n_az, elev))
    return pts, np.zeros(3)


def thin_wall_pair(seed=1, thickness=0.1, noise=0.01):
    """Two raw 64-ring frames on opposite sides of a thin partition wall.

    A 20 x 20 m room (3 m perimeter walls), a partition 5 m long, `thickness`
    thick and 2.5 m high whose faces lie inside one voxel of 0.25/0.5/1 m
    (centre plane y = 0.35 m), and ten 2-3 m boxes away from the partition.
    Sensor A (the target) sits 2 m south of the partition, sensor B (the
    source) 2.5 m north, both at 1.2 m height; each sees only its own face of
    the partition.  Returns (points_A, points_B) in their sensor frames, the
    relative pose T_A^-1 T_B and the sensors' world poses.
    """
    scene_rng, noise_rng = (np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(2))
    W, th, H = 10.0, 0.3, 3.0
    lo = [[-W - th, -W - th, 0], [W, -W - th, 0], [-W - th, -W - th, 0], [-W - th, W, 0],
          [-2.5, 0.35 - thickness / 2, 0]]
    hi = [[-W, W + th, H], [W + th, W + th, H], [W + th, -W, H], [W + th, W + th, H],
          [2.5, 0.35 + thickness / 2, 2.5]]
    for _ in range(10):
        c = scene_rng.uniform(-8, 8, 2)
        while abs(c[1]) < 4.5 and abs(c[0]) < 4.5:
            c = scene_rng.uniform(-8, 8, 2)
        sz = scene_rng.uniform(2.0, 3.0, 2)
        h = scene_rng.uniform(0.5, 2.5)
        lo.append([c[0] - sz[0] / 2, c[1] - sz[1] / 2, 0])
        hi.append([c[0] + sz[0] / 2, c[1] + sz[1] / 2, h])
    lo, hi = np.array(lo, float), np.array(hi, float)
    dirs = _lidar_dirs(64, 1024, (-30.0, 30.0))
    TA = yaw_pose(0.0, -2.0, 1.2, 0.3)
    TB = yaw_pose(0.5, 2.5, 1.2, -0.4)
    pa = lidar_frame(noise_rng, TA, lo, hi, dirs, rmin=0.5, rmax=40.0, noise=noise)
    pb = lidar_frame(noise_rng, TB, lo, hi, dirs, rmin=0.5, rmax=40.0, noise=noise)
    return {"target_raw": pa, "source_raw": pb, "T_true": inv_pose(TA) @ TB, "T_A": TA, "T_B": TB,
            "wall": (lo[4], hi[4])}


def local_mapping(seed=8, n_frames=15, spacing=1.0, n_rings=64, n_az=1024, angle_deg=0.5, trans_m=0.05):
    """Local-mapping submap (Sec. V-A): n_frames raw 64-ring frames along a
    trajectory in the urban block, `spacing` metres apart, matched all-to-all:
    one factor per pair i < j (source frame i into target frame j), 105 for 15
    frames.  Frame poses are estimates = truth (x) a seeded (angle_deg,
    trans_m) error per frame.  Raw points are in each sensor frame (the
    preprocessing input); the sensor sits at each frame's origin."""
    scene_rng, traj_rng, noise_rng, pose_rng = (np.random.default_rng(s) for s in
                                                np.random.SeedSequence(seed).spawn(4))
    s, x, y, yaw = _smooth_trajectory(traj_rng, float((n_frames - 1) * spacing))
    lo, hi = _urban_scene(scene_rng, np.stack([x, y], axis=1))
    dirs = _lidar_dirs(n_rings, n_az, (-22.5, 22.5))
    truth, est, raw = [], [], []
    for f in range(n_frames):
        i = int(round(f * spacing / (s[1] - s[0])))
        T = yaw_pose(x[i], y[i], 1.8, yaw[i])
        truth.append(T)
        est.append(T @ random_pose(pose_rng, angle_deg, trans_m))
        raw.append(lidar_frame(noise_rng, T, lo, hi, dirs))
    pairs = [(i, j) for i in range(n_frames) for j in range(i + 1, n_frames)]
    return {"raw": raw, "poses_true": truth, "poses_est": est, "pairs": pairs,
            "rel_est": [inv_pose(est[j]) @ est[i] for (i, j) in pairs],
            "rel_true": [inv_pose(truth[j]) @ truth[i] for (i, j) in pairs]}


def config2(seed=2, n_keyframes=20, resolutions=(0.25, 0.5, 1.0, 2.0), n_rings=32, n_az=1000,
            workers=-1):
    """One new 32-ring frame matched against 20 keyframes spaced 1 m apart (4-level maps)."""
    scene_rng, traj_rng, noise_rng, pose_rng = (np.random.default_rng(s) for s in
                                                np.random.SeedSequence(seed).spawn(4))
    s, x, y, yaw = _smooth_trajectory(traj_rng, float(n_keyframes))
    lo, hi = _urban_scene(scene_rng, np.stack([x, y], axis=1))
    dirs = _lidar_dirs(n_rings, n_az)
    poses = []
    for k in range(n_keyframes + 1):
        i = int(round(k / (s[1] - s[0])))
        poses.append(yaw_pose(x[i], y[i], 1.8, yaw[i]))
    snap = max(resolutions)
    clouds = []
    for k in range(n_keyframes + 1):
        pts = lidar_frame(noise_rng, poses[k], lo, hi, dirs)
        clouds.append(make_cloud(pts, np.zeros(3), snap, workers=workers))
    new = n_keyframes
    err = random_pose(pose_rng, 1.0, 0.1)
    T_new_est = poses[new] @ err
    rel = [inv_pose(poses[k]) @ T_new_est for k in range(n_keyframes)]
    rel_true = [inv_pose(poses[k]) @ poses[new] for k in range(n_keyframes)]
    return {
        "name": "odometry batch",
        "targets": clouds[:n_keyframes],
        "sources": [clouds[new]],
        "resolutions": list(resolutions),
        "factors": [(0, k) for k in range(n_keyframes)],
        "poses": rel,
        "poses_true": rel_true,
        "target_viewpoints": [np.zeros(3)] * n_keyframes,
    }


# ----------------------------------------------------------------------------
# config 3: global submap batch along a closed loop

TILE = 40.0


class Config3Layout:
    """Loop geometry, submap poses and sizes of the global batch (cheap to build)."""

    def __init__(self, seed=3, n_submaps=500, frames_per_submap=10, n_range=(50_000, 300_000),
                 corridor=60.0, sensor_range=45.0, resolution=0.5, k_range=(3, 7)):
        self.seed = seed
        self.n_submaps = n_submaps
        self.fps = frames_per_submap
        self.corridor = corridor
        self.sensor_range = sensor_range
        self.resolution = resolution
        self.k_range = k_range
        rng_loop, rng_n, rng_err = (np.random.default_rng(s) for s in
                                    np.random.SeedSequence([seed, 0]).spawn(3))
        length = float(n_submaps * frames_per_submap)
        phi = np.linspace(0, 2 * math.pi, 200_001)
        p1, p2 = rng_loop.uniform(0, 2 * math.pi, 2)
        a1, a2 = rng_loop.uniform(0.01, 0.03, 2)
        shape = 1.0 + a1 * np.sin(2 * phi + p1) + a2 * np.sin(3 * phi + p2)
        R0 = length / (2 * math.pi)
        for _ in range(3):
            px, py = R0 * shape * np.cos(phi), R0 * shape * np.sin(phi)
            seg = np.hypot(np.diff(px), np.diff(py))
            R0 *= length / seg.sum()
        px, py = R0 * shape * np.cos(phi), R0 * shape * np.sin(phi)
        arc = np.concatenate([[0.0], np.cumsum(np.hypot(np.diff(px), np.diff(py)))])
        n_frames = n_submaps * frames_per_submap
        sf = np.arange(n_frames, dtype=np.float64) * (arc[-1] / n_frames)
        fx = np.interp(sf, arc, px)
        fy = np.interp(sf, arc, py)
        eps = 0.05
        gx = np.interp((sf + eps) % arc[-1], arc, px) - np.interp((sf - eps) % arc[-1], arc, px)
        gy = np.interp((sf + eps) % arc[-1], arc, py) - np.interp((sf - eps) % arc[-1], arc, py)
        self.frame_xy = np.stack([fx, fy], axis=1)
        self.frame_yaw = np.arctan2(gy, gx)
        dense = np.stack([np.interp(np.arange(0, arc[-1], 1.0), arc, px),
                          np.interp(np.arange(0, arc[-1], 1.0), arc, py)], axis=1)
        self.loop_pts = dense
        c = np.arange(n_submaps) * frames_per_submap + frames_per_submap // 2
        self.centre_pose = [yaw_pose(fx[j], fy[j], 1.8, self.frame_yaw[j]) for j in c]
        ln = rng_n.uniform(math.log(n_range[0]), math.log(n_range[1]), n_submaps)
        self.n_points = np.round(np.exp(ln)).astype(np.int64)
        self.est_pose = [T @ random_pose(rng_err, 0.5, 0.1) for T in self.centre_pose]

    def factors(self):
        out = []
        k0, k1 = self.k_range
        for i in range(self.n_submaps):
            for sgn in (+1, -1):
                for k in range(k0, k1 + 1):
                    out.append((i, (i + sgn * k) % self.n_submaps))
        return out

    def tile_boxes(self, tx, ty, loop_tree):
        rng = _rng(self.seed, 1_000_003 + tx, 1_000_003 + ty)
        cx, cy = TILE * tx, TILE * ty
        lo, hi = random_boxes(rng, 20, (cx - 17.5, cy - 17.5), (cx + 17.5, cy + 17.5), 1.0, 5.0)
        keep = []
        for b in range(lo.shape[0]):
            c = (lo[b, :2] + hi[b, :2]) / 2
            half = (hi[b, :2] - lo[b, :2]) / 2
            near = loop_tree.query_ball_point(c, float(np.linalg.norm(half)) + 4.0)
            if near:
                d = np.maximum(np.abs(self.loop_pts[near] - c) - half, 0.0)
                if np.min(np.linalg.norm(d, axis=1)) < 3.0:
                    continue
            keep.append(b)
        return lo[keep], hi[keep]


def config3_submap(layout: Config3Layout, i: int, workers: int = 1) -> Cloud:
    """Submap i: visible surfaces within range of its 10 frames, in its centre frame."""
    rng = _rng(layout.seed, 7, i)
    loop_tree = cKDTree(layout.loop_pts)
    fr = np.arange(i * layout.fps, (i + 1) * layout.fps)
    fxy = layout.frame_xy[fr]
    rr = layout.sensor_range
    lo_xy = fxy.min(axis=0) - rr
    hi_xy = fxy.max(axis=0) + rr
    t0 = np.floor((lo_xy + TILE / 2) / TILE).astype(int)
    t1 = np.floor((hi_xy + TILE / 2) / TILE).astype(int)
    tiles = [(tx, ty) for tx in range(t0[0], t1[0] + 1) for ty in range(t0[1], t1[1] + 1)]

    def accept(p):
        d = np.min(np.linalg.norm(p[:, None, :2] - fxy[None], axis=2), axis=1)
        ok = d <= rr
        if ok.any():
            dc, _ = loop_tree.query(p[ok, :2], workers=workers)
            sub = dc <= layout.corridor
            ok[np.nonzero(ok)[0][~sub]] = False
        return ok

    need = int(layout.n_points[i])
    tile_data = []
    for (tx, ty) in tiles:
        lo, hi = layout.tile_boxes(tx, ty, loop_tree)
        area = TILE * TILE + float(np.sum((hi - lo)[:, 0] * (hi - lo)[:, 1]
                                          + 2 * (hi - lo)[:, 2] * ((hi - lo)[:, 0] + (hi - lo)[:, 1])))
        tile_data.append((tx, ty, lo, hi, area))
    tot_area = sum(t[4] for t in tile_data)
    got = []
    have = 0
    mult = 2.5
    while have < need:
        for (tx, ty, lo, hi, area) in tile_data:
            m = int(math.ceil(mult * need * area / tot_area)) + 16
            cx, cy = TILE * tx, TILE * ty
            p = sample_surfaces(rng, lo, hi, (cx - TILE / 2, cy - TILE / 2),
                                (cx + TILE / 2, cy + TILE / 2), m, noise=0.0, batch=m)
            p = p[accept(p)]
            got.append(p)
            have += p.shape[0]
        mult = 1.0
    pts = np.concatenate(got, axis=0)
    sel = rng.choice(pts.shape[0], need, replace=False)
    pts = pts[np.sort(sel)]
    pts = pts + rng.normal(0.0, 0.02, pts.shape)
    Tc = layout.centre_pose[i]
    local = apply_pose(inv_pose(Tc), pts)
    return make_cloud(local, np.zeros(3), layout.resolution, workers=workers)


def _submap_worker(args):
    layout, i = args
    return config3_submap(layout, i, workers=1)


def config3_factor_list(layout: Config3Layout):
    """(source, target) submap pairs and the relative poses they are linearized at."""
    fac = layout.factors()
    poses = [inv_pose(layout.est_pose[t]) @ layout.est_pose[s] for (s, t) in fac]
    poses_true = [inv_pose(layout.centre_pose[t]) @ layout.centre_pose[s] for (s, t) in fac]
    return fac, poses, poses_true


def config3(seed=3, n_submaps=500, n_range=(50_000, 300_000), processes=None, submaps=None):
    """Global batch: 500 submaps (50k-300k points, log-uniform), 5,000 directed factors.

    Submap i is the source of factors to submaps (i +- k) mod n, k = 3..7.
    ``submaps`` restricts generation to a subset of submap indices (others None).
    """
    layout = Config3Layout(seed=seed, n_submaps=n_submaps, n_range=n_range)
    idx = list(range(n_submaps)) if submaps is None else sorted(set(submaps))
    procs = processes or min(16, os.cpu_count() or 1)
    clouds = [None] * n_submaps
    if procs > 1 and len(idx) > 1:
        with ProcessPoolExecutor(procs) as ex:
            for i, c in zip(idx, ex.map(_submap_worker, [(layout, i) for i in idx], chunksize=1)):
                clouds[i] = c
    else:
        for i in idx:
            clouds[i] = config3_submap(layout, i, workers=-1)
    fac, poses, poses_true = config3_factor_list(layout)
    return {
        "name": "global submap batch",
        "layout": layout,
        "targets": clouds,
        "sources": clouds,
        "resolutions": [layout.resolution],
        "factors": fac,
        "poses": poses,
        "poses_true": poses_true,
        "target_viewpoints": [np.zeros(3)] * len(fac),
    }


# ----------------------------------------------------------------------------
# tiny exact cases


def tiny_lattice_pair(seed, n_cells=(6, 6, 3), r_max=1.0, margin=0.1, resolutions=(0.25, 0.5, 1.0)):
    """One point per coarse voxel, every other cell, offsets kept ``margin`` from faces.

    With source == target and T = identity every point sits alone in its voxel
    at every level, so the voxel mean equals the point and the residual is 0.
    Covariances are random SPD (float32-exact).
    """
    rng = _rng(11, seed)
    ii = np.stack(np.meshgrid(*[np.arange(0, 2 * n, 2) for n in n_cells], indexing="ij"), axis=-1).reshape(-1, 3)
    ii = ii - np.array(n_cells)  # include negative cells
    off = rng.uniform(margin, r_max - margin, ii.shape)
    xyz = (ii * r_max + off).astype(np.float32).astype(np.float64)
    A = rng.normal(size=(xyz.shape[0], 3, 3))
    C = np.einsum("nij,nkj->nik", A, A) + 0.05 * np.eye(3)[None]
    cov = np.stack([C[:, 0, 0], C[:, 0, 1], C[:, 0, 2], C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]], axis=1)
    cov = cov.astype(np.float32).astype(np.float64)
    nrm = rng.normal(size=xyz.shape)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    cloud = Cloud(np.zeros(3), xyz.astype(np.float32), cov.astype(np.float32),
                  nrm.astype(np.float32), np.zeros(3))
    return cloud, list(resolutions)
