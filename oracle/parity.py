"""Comparison of device results with the FP64 oracle (test infrastructure).

Correspondences: voxel keys must be bit-identical except for points whose FP64
transformed position lies within ``band`` (1e-5 m) of a face of its voxel;
those are counted, and for them either neighbouring voxel is a correct answer.
The expected e/H/b is the oracle's, with the contribution of every such point
whose device key differs replaced by the oracle's own terms for the device's
key (both terms come from the oracle).

Relative errors: e |e - e*| / |e*|, H ||H - H*||_F / ||H*||_F, b ||b - b*|| / ||b*||,
and, because a whole-matrix norm is dominated by the rotation block (lever arms
of metres), each block against its own scale as well: H_ww, H_wv, H_vv (3x3
blocks, Frobenius) and the diagonally scaled error
max_ij |H_ij - H*_ij| / sqrt(H*_ii H*_jj).  The halves of b (b_w rotation,
b_v translation) are sums whose summands cancel, strongly so near convergence,
so their errors are stated against the scale of those summands: the sum over
matched pairs of |b_k| of that half (the oracle's gradient_scale); their errors
against their own norms are reported beside them (b_w_own, b_v_own).
"""

from __future__ import annotations

import numpy as np

BAND = 1e-5
REL = 1e-5


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return 0.0 if np.linalg.norm(a) == 0.0 else np.inf
    return float(np.linalg.norm(a - b) / nb)


def block_errors(H_dev, b_dev, H, b, b_scale=None):
    """Relative errors of the blocks of H (rotation first), each against its own
    norm, the diagonally scaled error of H, and the errors of the halves of b:
    against their own norms (b_w_own, b_v_own) and, when ``b_scale`` (the
    oracle's gradient_scale) is given, against the scale of their summands
    (b_w, b_v)."""
    H_dev, b_dev, H, b = (np.asarray(x, dtype=np.float64) for x in (H_dev, b_dev, H, b))
    d = np.sqrt(np.abs(np.diag(H)))
    scale = np.outer(d, d)
    with np.errstate(divide="ignore", invalid="ignore"):
        hs = np.where(scale > 0, np.abs(H_dev - H) / scale, np.where(H_dev == H, 0.0, np.inf))
    out = {"H_ww": rel_err(H_dev[:3, :3], H[:3, :3]), "H_wv": rel_err(H_dev[:3, 3:], H[:3, 3:]),
           "H_vv": rel_err(H_dev[3:, 3:], H[3:, 3:]), "H_scaled": float(np.max(hs)) if hs.size else 0.0,
           "b_w_own": rel_err(b_dev[:3], b[:3]), "b_v_own": rel_err(b_dev[3:], b[3:])}
    if b_scale is not None:
        for name, sl, sc in (("b_w", slice(0, 3), b_scale[0]), ("b_v", slice(3, 6), b_scale[1])):
            num = float(np.linalg.norm(b_dev[sl] - b[sl]))
            out[name] = 0.0 if num == 0.0 else (num / sc if sc > 0 else np.inf)
    return out


ASSERTED = ("e", "H", "b", "H_ww", "H_wv", "H_vv", "H_scaled", "b_w", "b_v")


def visibility_margin(ofac, pose):
    """|(mu - T^-1 c) . n| per point, FP64 (the quantity the visibility rule thresholds at 0)."""
    T = np.asarray(pose)
    R, t = T[:3, :3], T[:3, 3]
    cs = R.T @ (ofac.viewpoint - t)
    return np.abs(np.einsum("ni,ni->n", ofac.xyz - cs[None], ofac.nrm))


def expected_with_device_keys(ofac, pose, keys_dev, found_dev, band=BAND, vis_band=1e-4):
    """Oracle e/H/b with ambiguous points resolved the way the device resolved them.

    Returns (e, H, b, stats) and asserts every unambiguous key is identical.
    """
    tr = ofac.linearize(pose, trace=True)
    keys_o, vidx_o, face, vis_o = tr["keys"], tr["vidx"], tr["face"], tr["visible"]
    n, L = vidx_o.shape
    e, H, b = tr["e"], tr["H"].copy(), tr["b"].copy()
    near = face < band
    mism = np.any(keys_dev != keys_o, axis=2)
    bad = mism & ~near
    assert not bad.any(), "device keys differ from the oracle away from voxel faces: %d cases, e.g. %s" % (
        int(bad.sum()), list(zip(*np.nonzero(bad)))[:5])
    # visibility: -1 from the device means discarded
    vis_dev = ~np.all(found_dev == -1, axis=1) if L else np.ones(n, bool)
    vis_flip = vis_dev != vis_o
    if vis_flip.any():
        marg = visibility_margin(ofac, pose)
        assert np.all(marg[vis_flip] < vis_band), "visibility differs away from the tie"
    # found flags must agree where keys agree and the point is visible on both sides
    both = vis_dev & vis_o
    fo = (vidx_o >= 0)
    fd = (found_dev == 1)
    same_key = ~mism
    agree = fo[both[:, None] & same_key] == fd[both[:, None] & same_key] if n else np.array([True])
    assert np.all(agree), "found flags differ for identical keys"
    adjusted = 0
    todo = np.nonzero(mism | vis_flip[:, None])
    for k, l in zip(*todo):
        own_used = vis_o[k] and vidx_o[k, l] >= 0
        dev_used = vis_dev[k] and found_dev[k, l] == 1
        if own_used:
            ok, e1, H1, b1 = ofac.point_terms(pose, k, l, keys_o[k, l])
            e -= e1
            H -= H1
            b -= b1
        if dev_used:
            ok, e2, H2, b2 = ofac.point_terms(pose, k, l, keys_dev[k, l])
            assert ok
            e += e2
            H += H2
            b += b2
        adjusted += 1
    stats = {"near_face": int(near.sum()), "near_face_mismatch": int((mism & near).sum()),
             "visibility_flips": int(vis_flip.sum()), "adjusted": adjusted,
             "inliers_oracle": tr["inliers"].tolist()}
    return e, H, b, stats


def check_factor(batch, f, pose, ofac, e_dev, H_dev, b_dev, rel=REL):
    """Device e/H/b of factor f against the oracle (face-band rule applied): the
    whole-matrix errors and every block error must be within `rel`."""
    keys_dev, found_dev = batch.correspondences(pose, f)
    e, H, b, stats = expected_with_device_keys(ofac, pose, keys_dev, found_dev)
    errs = {"e": rel_err(e_dev, e), "H": rel_err(H_dev, H), "b": rel_err(b_dev, b)}
    errs.update(block_errors(H_dev, b_dev, H, b, ofac.gradient_scale(pose)))
    assert max(errs[k] for k in ASSERTED) <= rel, (errs, stats)
    return errs, stats


def _packed(vmap, level):
    """Voxel keys of an oracle level packed into one int64 each, in the same (lexicographic) order."""
    cache = vmap.__dict__.setdefault("_packed_keys", {})
    if level not in cache:
        k = vmap.levels[level][0]
        cache[level] = ((k[:, 0] + (1 << 20)) << 42) | ((k[:, 1] + (1 << 20)) << 21) | (k[:, 2] + (1 << 20))
    return cache[level]


def oracle_voxel_index(vmap, level, key):
    """Index of voxel `key` in the oracle's level (lexicographic order), -1 if absent."""
    pk = _packed(vmap, level)
    q = ((int(key[0]) + (1 << 20)) << 42) | ((int(key[1]) + (1 << 20)) << 21) | (int(key[2]) + (1 << 20))
    i = int(np.searchsorted(pk, q))
    return i if i < len(pk) and pk[i] == q else -1


def frozen_from_device_keys(ofac, pose, keys_dev, found_dev, band=BAND):
    """Per point and level, the oracle voxel index of the device's correspondence
    (-1 where the device found none or discarded the point), for the oracle's
    frozen-correspondence evaluate / gradient.  Asserts that keys agree away
    from the face band."""
    tr = ofac.linearize(pose, trace=True)
    keys_o, vidx_o, face = tr["keys"], tr["vidx"], tr["face"]
    mism = np.any(keys_dev != keys_o, axis=2)
    assert not (mism & ~(face < band)).any(), "device keys differ from the oracle away from voxel faces"
    fz = vidx_o.copy()
    fz[found_dev != 1] = -1
    for k, l in zip(*np.nonzero(mism & (found_dev == 1))):
        fz[k, l] = oracle_voxel_index(ofac.vmap, l, keys_dev[k, l])
        assert fz[k, l] >= 0
    same = ~mism & (found_dev == 1)
    assert np.all(vidx_o[same] >= 0), "device found a voxel the oracle does not have"
    return fz, int(mism.sum())

