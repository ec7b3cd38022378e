"""Box-world scenes: area-uniform surface sampling and a spinning-LiDAR ray caster.

A scene is a ground plane z = 0 plus axis-aligned boxes resting on it.  The
visible surfaces are the ground outside the box footprints and every box's top
and four sides; a sample that falls strictly inside another box is hidden.
"""

from __future__ import annotations

import numpy as np


def random_boxes(rng, n, centre_lo, centre_hi, side_lo, side_hi, height_lo=None, height_hi=None):
    """(lo, hi) corner arrays of n axis-aligned boxes resting on z = 0."""
    cx = rng.uniform(centre_lo[0], centre_hi[0], n)
    cy = rng.uniform(centre_lo[1], centre_hi[1], n)
    sx = rng.uniform(side_lo, side_hi, n)
    sy = rng.uniform(side_lo, side_hi, n)
    if height_lo is None:
        sz = rng.uniform(side_lo, side_hi, n)
    else:
        sz = rng.uniform(height_lo, height_hi, n)
    lo = np.stack([cx - sx / 2, cy - sy / 2, np.zeros(n)], axis=1)
    hi = np.stack([cx + sx / 2, cy + sy / 2, sz], axis=1)
    return lo, hi


def _inside_any(p, lo, hi, exclude=None):
    """Mask of points strictly inside any box (optionally ignoring box `exclude[i]` for point i)."""
    out = np.zeros(p.shape[0], dtype=bool)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    for b in range(lo.shape[0]):
        m = ((x > lo[b, 0]) & (x < hi[b, 0]) & (y > lo[b, 1]) & (y < hi[b, 1])
             & (z > lo[b, 2]) & (z < hi[b, 2]))
        if exclude is not None:
            m &= exclude != b
        out |= m
    return out


def _in_footprint(p, lo, hi):
    out = np.zeros(p.shape[0], dtype=bool)
    x, y = p[:, 0], p[:, 1]
    for b in range(lo.shape[0]):
        out |= (x >= lo[b, 0]) & (x <= hi[b, 0]) & (y >= lo[b, 1]) & (y <= hi[b, 1])
    return out


def sample_surfaces(rng, lo, hi, ground_lo, ground_hi, n, noise=0.02, accept=None, batch=None):
    """Area-uniform samples on the visible surfaces, with isotropic Gaussian noise.

    ``accept`` is an optional mask function on noise-free candidates (e.g. a
    visibility-range region).  Returns exactly n points (float64, (n, 3)).
    """
    B = lo.shape[0]
    size = hi - lo
    g_area = (ground_hi[0] - ground_lo[0]) * (ground_hi[1] - ground_lo[1])
    # faces: 0 ground; per box: top, -x, +x, -y, +y
    areas = [g_area]
    for b in range(B):
        sx, sy, sz = size[b]
        areas += [sx * sy, sy * sz, sy * sz, sx * sz, sx * sz]
    areas = np.asarray(areas)
    prob = areas / areas.sum()
    got = []
    total = 0
    batch = batch or max(4096, 2 * n)
    while total < n:
        f = rng.choice(areas.shape[0], size=batch, p=prob)
        u = rng.random((batch, 2))
        p = np.empty((batch, 3))
        own = np.full(batch, -1, dtype=np.int64)
        g = f == 0
        p[g, 0] = ground_lo[0] + u[g, 0] * (ground_hi[0] - ground_lo[0])
        p[g, 1] = ground_lo[1] + u[g, 1] * (ground_hi[1] - ground_lo[1])
        p[g, 2] = 0.0
        bf = ~g
        b = (f[bf] - 1) // 5
        face = (f[bf] - 1) % 5
        blo, bhi = lo[b], hi[b]
        uu = u[bf]
        q = np.empty((b.shape[0], 3))
        # top
        t = face == 0
        q[t, 0] = blo[t, 0] + uu[t, 0] * (bhi[t, 0] - blo[t, 0])
        q[t, 1] = blo[t, 1] + uu[t, 1] * (bhi[t, 1] - blo[t, 1])
        q[t, 2] = bhi[t, 2]
        # -x / +x
        for fi, xval in ((1, blo[:, 0]), (2, bhi[:, 0])):
            t = face == fi
            q[t, 0] = xval[t]
            q[t, 1] = blo[t, 1] + uu[t, 0] * (bhi[t, 1] - blo[t, 1])
            q[t, 2] = blo[t, 2] + uu[t, 1] * (bhi[t, 2] - blo[t, 2])
        # -y / +y
        for fi, yval in ((3, blo[:, 1]), (4, bhi[:, 1])):
            t = face == fi
            q[t, 1] = yval[t]
            q[t, 0] = blo[t, 0] + uu[t, 0] * (bhi[t, 0] - blo[t, 0])
            q[t, 2] = blo[t, 2] + uu[t, 1] * (bhi[t, 2] - blo[t, 2])
        p[bf] = q
        own[bf] = b
        if accept is not None:
            sel = accept(p)
            p, own, g = p[sel], own[sel], g[sel]
        keep = np.ones(p.shape[0], dtype=bool)
        keep[g] = ~_in_footprint(p[g], lo, hi)
        keep &= ~_inside_any(p, lo, hi, exclude=own)
        p = p[keep]
        got.append(p)
        total += p.shape[0]
    pts = np.concatenate(got, axis=0)[:n]
    return pts + rng.normal(0.0, noise, pts.shape)


def _box_azimuth_ranges(origin, lo, hi):
    """Azimuth interval (centre, half-width) subtended by each box footprint from origin."""
    cx = (lo[:, 0] + hi[:, 0]) / 2 - origin[0]
    cy = (lo[:, 1] + hi[:, 1]) / 2 - origin[1]
    centre = np.arctan2(cy, cx)
    half = np.full(lo.shape[0], np.pi)
    for xs in (lo[:, 0], hi[:, 0]):
        for ys in (lo[:, 1], hi[:, 1]):
            a = np.arctan2(ys - origin[1], xs - origin[0])
            d = np.abs((a - centre + np.pi) % (2 * np.pi) - np.pi)
            half = np.where(half == np.pi, d, np.maximum(half, d))
    inside = ((origin[0] >= lo[:, 0]) & (origin[0] <= hi[:, 0])
              & (origin[1] >= lo[:, 1]) & (origin[1] <= hi[:, 1]))
    half[inside] = np.pi
    return centre, half


def raycast(origin, dirs, lo, hi, t_max=1e9):
    """Nearest hit distance of rays (origin + t*dir) against ground z=0 and boxes; inf if none."""
    n = dirs.shape[0]
    best = np.full(n, np.inf)
    dz = dirs[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = -origin[2] / dz
    ok = (dz < 0) & (tg > 0)
    best[ok] = tg[ok]
    if lo.shape[0]:
        az = np.arctan2(dirs[:, 1], dirs[:, 0])
        order = np.argsort(az, kind="stable")
        bc, bh = _box_azimuth_ranges(origin, lo, hi)
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / dirs
        step = 2048
        for s in range(0, n, step):
            idx = order[s:s + step]
            a0, a1 = az[idx[0]], az[idx[-1]]
            wc, wh = (a0 + a1) / 2, (a1 - a0) / 2
            dist = np.abs((bc - wc + np.pi) % (2 * np.pi) - np.pi)
            cand = np.nonzero(dist <= bh + wh + 1e-9)[0]
            if cand.size == 0:
                continue
            blo, bhi = lo[cand], hi[cand]
            iv = inv[idx][:, None, :]
            t1 = (blo[None] - origin[None, None, :]) * iv
            t2 = (bhi[None] - origin[None, None, :]) * iv
            t1 = np.nan_to_num(t1, nan=-np.inf)
            t2 = np.nan_to_num(t2, nan=np.inf)
            tmin = np.minimum(t1, t2).max(axis=2)
            tmax = np.maximum(t1, t2).min(axis=2)
            hit = (tmax >= tmin) & (tmax > 0) & (tmin > 0)
            tt = np.where(hit, tmin, np.inf).min(axis=1)
            best[idx] = np.minimum(best[idx], tt)
    best[best > t_max] = np.inf
    return best
