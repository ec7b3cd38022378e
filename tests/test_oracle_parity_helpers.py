"""The parity helpers (oracle/parity.py) on the oracle alone: with the oracle's own
correspondences the frozen evaluation reproduces the free one, and a key moved
to a neighbouring voxel resolves to that voxel's index."""

import numpy as np

import oracle
import synth
from oracle.parity import frozen_from_device_keys, oracle_voxel_index


def test_frozen_from_own_keys_reproduces_the_gradient():
    cfg = synth.config1(seed=5, n_target=6000, n_source=2000)
    of = oracle.factor_from_clouds(cfg["sources"][0], cfg["targets"][0], cfg["resolutions"])
    pose = cfg["poses_true"][0]
    tr = of.linearize(pose, trace=True)
    found = np.where(tr["vidx"] >= 0, 1, 0).astype(np.int32)
    fz, n_face = frozen_from_device_keys(of, pose, tr["keys"], found)
    assert n_face == 0
    assert np.array_equal(fz, tr["vidx"])
    g0, gm0 = of.gradient(pose)
    g1, gm1 = of.gradient(pose, frozen=fz)
    np.testing.assert_array_equal(g0, g1)
    np.testing.assert_array_equal(gm0, gm1)


def test_voxel_index_lookup():
    cfg = synth.config1(seed=6, n_target=3000, n_source=10)
    vm = oracle.VoxelMap(cfg["targets"][0].xyz64(), cfg["targets"][0].cov64(), [0.5, 1.0])
    for level in (0, 1):
        keys = vm.levels[level][0]
        for v in (0, len(keys) // 2, len(keys) - 1):
            assert oracle_voxel_index(vm, level, keys[v]) == v
        assert oracle_voxel_index(vm, level, keys.max(axis=0) + 5) == -1


# ---------------------------------------------------------------- face-band adjustment pins

import pytest

from oracle.parity import BAND, expected_with_device_keys


def _case(seed=7, n_target=8000, n_source=2500, res=(0.5,)):
    cfg = synth.config1(seed=seed, n_target=n_target, n_source=n_source, resolutions=res)
    of = oracle.factor_from_clouds(cfg["sources"][0], cfg["targets"][0], cfg["resolutions"])
    return cfg, of, np.asarray(cfg["poses"][0], dtype=np.float64)


def _found(tr):
    """Device-style found flags from an oracle trace: 1 voxel, 0 none, -1 discarded."""
    f = np.where(tr["vidx"] >= 0, 1, 0).astype(np.int32)
    f[~tr["visible"]] = -1
    return f


def test_own_keys_reproduce_linearize_bit_for_bit():
    """Handed the oracle's own keys, the adjusted expectation is the oracle's result, unchanged."""
    for res in ((0.5,), (0.25, 0.5, 1.0)):
        cfg, of, pose = _case(res=res)
        tr = of.linearize(pose, trace=True)
        e, H, b, stats = expected_with_device_keys(of, pose, tr["keys"], _found(tr))
        assert stats["adjusted"] == 0
        assert e == tr["e"] and np.array_equal(H, tr["H"]) and np.array_equal(b, tr["b"])


def test_point_terms_sum_to_linearize():
    """orc_point_terms of every (point, level) at the point's own key add up to orc_linearize,
    and a key with no voxel reports 0 with zero terms."""
    cfg, of, pose = _case(n_source=600, res=(0.5, 1.0))
    tr = of.linearize(pose, trace=True)
    e, H, b = 0.0, np.zeros((6, 6)), np.zeros(6)
    n_hit = 0
    for k in range(of.n):
        for l in range(of.vmap.L):
            ok, e1, H1, b1 = of.point_terms(pose, k, l, tr["keys"][k, l])
            assert ok == (tr["vidx"][k, l] >= 0)
            if not ok:
                assert e1 == 0.0 and not H1.any() and not b1.any()
            e += e1
            H += H1
            b += b1
            n_hit += ok
    assert n_hit == int(tr["inliers"].sum()) > 100
    assert abs(e - tr["e"]) <= 1e-12 * abs(tr["e"])
    np.testing.assert_allclose(H, tr["H"], rtol=0, atol=1e-12 * np.abs(tr["H"]).max())
    np.testing.assert_allclose(b, tr["b"], rtol=0, atol=1e-12 * np.abs(b).max())
    far = tr["keys"][0, 0] + np.array([10 ** 6, 0, 0])
    ok, e1, H1, b1 = of.point_terms(pose, 0, 0, far)
    assert not ok and e1 == 0.0 and not H1.any() and not b1.any()


def _moved_to_face(of, pose, k, axis, upper, gap=2e-7):
    """Move source point k so that its transformed position lies `gap` metres inside the
    upper (or lower) face of its voxel along `axis` at level 0; returns the new factor."""
    R, t = pose[:3, :3], pose[:3, 3]
    r = of.vmap.resolutions[0]
    y = R @ of.xyz[k] + t
    q = np.floor(y / r)
    y2 = y.copy()
    y2[axis] = (q[axis] + 1) * r - gap if upper else q[axis] * r + gap
    xyz = of.xyz.copy()
    xyz[k] = R.T @ (y2 - t)
    return oracle.Factor(xyz, of.cov, of.vmap, nrm=of.nrm, viewpoint=of.viewpoint, validate=of.validate)


def test_in_band_point_on_the_neighbouring_voxel_equals_frozen_linearize():
    """A point moved to within the band of a face, reported by the 'device' in the voxel across
    that face, gives the oracle's linearize with that point frozen to the neighbour (or to no
    voxel when the neighbour is empty) -- computed by a different route, so equal to rounding."""
    cfg, of0, pose = _case(n_source=3000)
    tr0 = of0.linearize(pose, trace=True)
    hits = np.nonzero(tr0["vidx"][:, 0] >= 0)[0]
    done = {"neighbour": 0, "empty": 0}
    rng = np.random.default_rng(3)
    for k in rng.permutation(hits):
        if min(done.values()) >= 2:
            break
        axis, upper = int(rng.integers(3)), bool(rng.integers(2))
        of = _moved_to_face(of0, pose, k, axis, upper)
        tr = of.linearize(pose, trace=True)
        assert tr["face"][k, 0] < BAND and tr["vidx"][k, 0] >= 0
        keys_dev = tr["keys"].copy()
        keys_dev[k, 0, axis] += 1 if upper else -1
        nb = oracle_voxel_index(of.vmap, 0, keys_dev[k, 0])
        kind = "neighbour" if nb >= 0 else "empty"
        if done[kind] >= 2:
            continue
        found_dev = _found(tr)
        found_dev[k, 0] = 1 if nb >= 0 else 0
        e, H, b, stats = expected_with_device_keys(of, pose, keys_dev, found_dev)
        assert stats["adjusted"] == 1 and stats["near_face_mismatch"] == 1
        fz = tr["vidx"].copy()
        fz[k, 0] = nb
        ref = of.linearize(pose, frozen=fz)
        assert abs(e - ref["e"]) <= 1e-11 * abs(ref["e"])
        np.testing.assert_allclose(H, ref["H"], rtol=0, atol=1e-11 * np.abs(ref["H"]).max())
        np.testing.assert_allclose(b, ref["b"], rtol=0, atol=1e-11 * np.abs(ref["b"]).max())
        # and the point's own terms did change the result (the test can tell them apart)
        assert abs(ref["e"] - tr["e"]) > 1e-9 * abs(tr["e"])
        done[kind] += 1
    assert done["neighbour"] >= 2 and done["empty"] >= 2, done


def test_key_change_outside_the_band_raises():
    cfg, of, pose = _case()
    tr = of.linearize(pose, trace=True)
    k = int(np.argmax(tr["face"][:, 0]))
    assert tr["face"][k, 0] > 100 * BAND
    keys_dev = tr["keys"].copy()
    keys_dev[k, 0, 1] += 1
    with pytest.raises(AssertionError, match="away from voxel faces"):
        expected_with_device_keys(of, pose, keys_dev, _found(tr))


def test_face_trace_is_the_distance_to_the_nearest_face():
    """Displacing y by just under the traced distance along any axis keeps its key; just over
    it, toward the nearest face, changes it (so the trace is neither too small nor too large)."""
    cfg, of, pose = _case(n_source=400, res=(0.25, 1.0))
    R, t = pose[:3, :3], pose[:3, 3]
    tr = of.linearize(pose, trace=True)
    Y = of.xyz @ R.T + t
    for l, r in enumerate(of.vmap.resolutions):
        for k in range(of.n):
            y, key, f = Y[k], tr["keys"][k, l], tr["face"][k, l]
            assert np.array_equal(np.floor(y / r).astype(np.int64), key)
            changed = []
            for a in range(3):
                for s in (-1.0, 1.0):
                    inside = y.copy()
                    inside[a] += s * f * (1 - 1e-6)
                    assert np.array_equal(np.floor(inside / r).astype(np.int64), key)
                    out = y.copy()
                    out[a] += s * (f * (1 + 1e-6) + 1e-12)
                    changed.append(not np.array_equal(np.floor(out / r).astype(np.int64), key))
            assert any(changed), (k, l, f)


def test_block_errors_see_what_whole_matrix_norms_hide():
    """A per-mille error in the translation block of H (or of b) is invisible in
    the whole-matrix relative error, which the rotation block dominates, but not
    in the block errors; an exact copy has every block error 0."""
    from oracle.parity import block_errors, rel_err
    cfg = synth.config1(seed=3, n_target=4000, n_source=1500)
    of = oracle.factor_from_clouds(cfg["sources"][0], cfg["targets"][0], cfg["resolutions"])
    r = of.linearize(cfg["poses"][0])
    H, b = r["H"], r["b"]
    assert max(block_errors(H, b, H, b).values()) == 0.0
    Hp = H.copy()
    Hp[3:, 3:] *= 1.0 + 2e-3
    errs = block_errors(Hp, b, H, b)
    assert errs["H_vv"] == pytest.approx(2e-3, rel=1e-6)
    assert errs["H_scaled"] >= 2e-3 * (1 - 1e-9)
    assert errs["H_ww"] == 0.0 and errs["H_wv"] == 0.0
    assert rel_err(Hp, H) < errs["H_vv"] / 10          # the whole-matrix norm hides most of it
    bp = b.copy()
    bp[3:] *= 1.0 + 2e-3
    sc = of.gradient_scale(cfg["poses"][0])
    errs = block_errors(H, bp, H, b, sc)
    assert errs["b_v_own"] == pytest.approx(2e-3, rel=1e-6) and errs["b_w_own"] == 0.0
    assert errs["b_v"] == pytest.approx(2e-3 * np.linalg.norm(b[3:]) / sc[1], rel=1e-6) and errs["b_w"] == 0.0
    # an off-diagonal entry is measured against the geometric mean of its diagonal entries
    Hq = H.copy()
    Hq[0, 5] += 1e-4 * np.sqrt(H[0, 0] * H[5, 5])
    assert block_errors(Hq, b, H, b)["H_scaled"] == pytest.approx(1e-4, rel=1e-9)


def test_gradient_scale_is_the_sum_of_per_point_norms():
    """gradient_scale = sum over matched (point, level) pairs of the norms of the
    two halves of each pair's b, summed here from the per-point terms (which are
    pinned to add up to the factor's b); it bounds |b| of each half."""
    cfg = synth.config1(seed=8, n_target=3000, n_source=300, resolutions=(0.5, 1.0))
    of = oracle.factor_from_clouds(cfg["sources"][0], cfg["targets"][0], cfg["resolutions"])
    pose = cfg["poses_true"][0]
    tr = of.linearize(pose, trace=True)
    sw = sv = 0.0
    bsum = np.zeros(6)
    for k in range(of.n):
        for l in range(2):
            if tr["vidx"][k, l] < 0:
                continue
            ok, _, _, bk = of.point_terms(pose, k, l, tr["keys"][k, l])
            assert ok
            sw += np.linalg.norm(bk[:3])
            sv += np.linalg.norm(bk[3:])
            bsum += bk
    gw, gv = of.gradient_scale(pose)
    assert gw == pytest.approx(sw, rel=1e-12) and gv == pytest.approx(sv, rel=1e-12)
    np.testing.assert_allclose(bsum, tr["b"], rtol=1e-9, atol=1e-9 * np.abs(tr["b"]).max())
    assert np.linalg.norm(tr["b"][:3]) <= gw and np.linalg.norm(tr["b"][3:]) <= gv
    # at the true pose the translation half cancels: |b_v| is a small part of its scale
    print("cancellation |b_v| / scale = %.3g" % (np.linalg.norm(tr["b"][3:]) / gv))
