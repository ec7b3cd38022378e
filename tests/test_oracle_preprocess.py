"""Pins of the preprocessing oracle (oracle/preprocess.py) against facts other than itself:
scipy's k-d tree, hand-built clouds with known answers, closed forms, invariants."""

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import preprocess as pp


def test_downsample_one_point_per_voxel_is_a_sort():
    rng = np.random.default_rng(0)
    keys = rng.choice(40, size=(200, 3)) - 20
    keys = np.unique(keys, axis=0)
    rng.shuffle(keys)
    r = 0.25
    pts = (keys + rng.uniform(0.05, 0.95, size=keys.shape)) * r
    c, k, cnt = pp.downsample(pts, r)
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    np.testing.assert_array_equal(c, pts[order])
    np.testing.assert_array_equal(k, keys[order])
    assert np.all(cnt == 1)


def test_downsample_by_hand():
    r = 1.0
    pts = np.array([[0.1, 0.2, 0.3], [0.5, 0.6, 0.7], [-0.5, 0.0, 0.0], [0.9, 0.8, 0.1], [-0.25, 0.5, 0.5]])
    c, k, cnt = pp.downsample(pts, r)
    np.testing.assert_array_equal(k, [[-1, 0, 0], [0, 0, 0]])
    np.testing.assert_array_equal(cnt, [2, 3])
    np.testing.assert_allclose(c[0], [-0.375, 0.25, 0.25], rtol=0, atol=1e-15)
    np.testing.assert_allclose(c[1], [1.5 / 3, 1.6 / 3, 1.1 / 3], rtol=0, atol=1e-15)


def test_downsample_centroids_inside_their_voxels_and_counts_sum():
    rng = np.random.default_rng(1)
    pts = rng.normal(size=(5000, 3)) * 3.0
    r = 0.5
    c, k, cnt = pp.downsample(pts, r)
    assert cnt.sum() == len(pts)
    assert np.all(c >= k * r - 1e-12) and np.all(c <= (k + 1) * r + 1e-12)
    # brute force: every voxel's mean over a membership scan
    for v in range(0, len(k), 97):
        m = np.all(np.floor(pts / r) == k[v], axis=1)
        np.testing.assert_allclose(c[v], pts[m].mean(axis=0), rtol=0, atol=1e-13)


def test_knn_matches_kdtree():
    rng = np.random.default_rng(2)
    P = rng.uniform(-5, 5, size=(700, 3))
    idx, d2 = pp.knn(P, 10)
    dd, ii = cKDTree(P).query(P, k=10)
    np.testing.assert_array_equal(idx, ii)
    np.testing.assert_allclose(np.sqrt(d2), dd, rtol=1e-12, atol=1e-14)
    assert np.all(idx[:, 0] == np.arange(len(P))) and np.all(d2[:, 0] == 0)


def test_knn_ties_by_index_and_short_clouds():
    # a 3x3x3 unit lattice: the centre has 6 neighbours at distance 1, tie-broken by index
    g = np.stack(np.meshgrid(*[np.arange(3.0)] * 3, indexing="ij"), -1).reshape(-1, 3)
    idx, d2 = pp.knn(g, 7, queries=[13])
    assert idx[0, 0] == 13
    np.testing.assert_array_equal(idx[0, 1:], [4, 10, 12, 14, 16, 22])
    np.testing.assert_array_equal(d2[0], [0, 1, 1, 1, 1, 1, 1])
    idx, d2 = pp.knn(g[:3], 5)
    assert np.all(idx[:, 3:] == -1) and np.all(np.isinf(d2[:, 3:]))


def test_covariance_and_normal_of_a_plane():
    rng = np.random.default_rng(3)
    n_true = np.array([1.0, 2.0, 2.0]) / 3.0
    u = np.cross(n_true, [0, 0, 1.0])
    u /= np.linalg.norm(u)
    v = np.cross(n_true, u)
    P = rng.uniform(-1, 1, size=(300, 1)) * u + rng.uniform(-1, 1, size=(300, 1)) * v + [5.0, 0, 0]
    sensor = np.array([5.0, 0, 0]) + 4.0 * n_true
    idx, _ = pp.knn(P, 10)
    C = pp.covariance(P, idx)
    Creg, nrm, w = pp.regularize(C, P, sensor)
    np.testing.assert_allclose(nrm, np.broadcast_to(n_true, nrm.shape), atol=1e-9)
    assert np.all(np.abs(w[:, 0]) < 1e-15 * 1e3)
    expect = np.eye(3) - (1 - pp.EPS) * np.outer(n_true, n_true)
    np.testing.assert_allclose(Creg, np.broadcast_to(expect, Creg.shape), atol=1e-9)
    # the sensor on the other side flips every normal
    _, nrm2, _ = pp.regularize(C, P, np.array([5.0, 0, 0]) - 4.0 * n_true)
    np.testing.assert_allclose(nrm2, -nrm, atol=1e-12)


def test_covariance_by_hand():
    P = np.array([[0.0, 0, 0], [2.0, 0, 0], [0.0, 4.0, 0], [2.0, 4.0, 0]])
    C = pp.covariance(P, np.array([[0, 1, 2, 3]]))
    np.testing.assert_allclose(C[0], np.diag([1.0, 4.0, 0.0]), atol=0)
    Creg, n, w = pp.regularize(C, P[:1], np.array([0, 0, 10.0]))
    np.testing.assert_allclose(n[0], [0, 0, 1.0])
    np.testing.assert_allclose(Creg[0], np.diag([1.0, 1.0, pp.EPS]), atol=1e-15)
    np.testing.assert_allclose(w[0], [0.0, 1.0, 4.0], atol=1e-15)


@pytest.mark.parametrize("seed", [4, 5])
def test_rigid_motion_equivariance(seed):
    rng = np.random.default_rng(seed)
    P = rng.uniform(-3, 3, size=(400, 3))
    P[:, 2] = 0.2 * np.sin(P[:, 0]) + 0.01 * rng.normal(size=len(P))
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.linalg.det(q))
    t = rng.normal(size=3)
    sensor = np.array([0, 0, 3.0])
    idx, _ = pp.knn(P, 10)
    idx2, _ = pp.knn(P @ q.T + t, 10)
    np.testing.assert_array_equal(idx, idx2)
    C = pp.covariance(P, idx)
    C2 = pp.covariance(P @ q.T + t, idx2)
    np.testing.assert_allclose(C2, q[None] @ C @ q.T[None], atol=1e-12)
    _, n1, _ = pp.regularize(C, P, sensor)
    _, n2, _ = pp.regularize(C2, P @ q.T + t, q @ sensor + t)
    np.testing.assert_allclose(n2, n1 @ q.T, atol=1e-8)


def test_knn_tree_equals_brute_force():
    rng = np.random.default_rng(6)
    P = rng.normal(size=(900, 3)) * [5.0, 5.0, 0.5]
    a_idx, a_d2 = pp.knn(P, 12)
    b_idx, b_d2 = pp.knn_tree(P, 12)
    np.testing.assert_array_equal(a_idx, b_idx)
    np.testing.assert_array_equal(a_d2, b_d2)
    a_idx, _ = pp.knn(P[:5], 8)
    b_idx, _ = pp.knn_tree(P[:5], 8)
    np.testing.assert_array_equal(a_idx, b_idx)
