"""Device preprocessing (downsampling, exact k-NN, covariances, normals) against the
FP64 oracle in oracle/preprocess.py, through the C ABI (needs an MI355X).

Bar: downsampled points and counts bit-exact (same FP64 sums in the same
order); neighbour indices and squared distances bit-exact (same rounded
operations, ties by index); raw covariances within 1e-11 of the largest
eigenvalue; normals and regularised covariances within a bound scaled by the
eigen-gap where the smallest eigenvector is well defined, otherwise checked
for validity (unit length, Rayleigh quotient at the smallest eigenvalue).
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import preprocess as pp
from oracle.parity import check_factor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    from paper_2407_10344_amd import vgicp
    ctx = vgicp.Context(0)
    yield vgicp, ctx
    ctx.close()


@pytest.fixture(scope="module")
def frame():
    return synth.raw_frame()


def device(vgicp, ctx, xyz, r, k, sensor):
    c = vgicp.Cloud(ctx, xyz, r, k, sensor)
    out = c.export()
    c.close()
    return out


def check_cov_normals(dev, rows, P, nbr_o, sensor):
    """Covariance / normal checks for cloud rows `rows` (oracle recomputed on its own neighbours)."""
    C = pp.covariance(P, nbr_o)
    Creg, n_o, w = pp.regularize(C, P[rows], sensor)
    lam = np.maximum(w[:, 2], 1e-300)
    craw = dev["cov_raw"][rows]
    err = np.abs(craw - pp.cov6(C)).max(axis=1)
    assert np.all(err <= 1e-11 * lam + 1e-18), err.max()
    n_d = dev["normals"][rows]
    assert np.allclose(np.linalg.norm(n_d, axis=1), 1.0, atol=1e-12)
    gap = (w[:, 1] - w[:, 0]) / lam
    well = gap > 1e-6
    tol = 1e-11 / np.maximum(gap, 1e-300) + 1e-12
    # orientation: the sign is fixed unless the normal is (almost) perpendicular to the sensor ray
    ray = sensor[None] - P[rows]
    marg = np.abs(np.einsum("ni,ni->n", n_o, ray)) / np.maximum(np.linalg.norm(ray, axis=1), 1e-300)
    sgn = np.where((marg < 1e-9) & (np.einsum("ni,ni->n", n_d, n_o) < 0), -1.0, 1.0)
    dn = np.linalg.norm(n_d - sgn[:, None] * n_o, axis=1)
    assert np.all(dn[well] <= tol[well]), (dn[well] / tol[well]).max()
    # ill-conditioned rows: any unit vector of the smallest eigen-space is correct
    M = np.stack([C[:, 0], C[:, 1], C[:, 2]], axis=1)
    rq = np.einsum("ni,nij,nj->n", n_d, M, n_d)
    assert np.all(rq[~well] <= w[~well, 0] + 1e-6 * lam[~well])
    creg_d = dev["cov"][rows]
    assert np.all(np.abs(creg_d - pp.cov6(Creg))[well].max(axis=1) <= 2 * tol[well] + 1e-15)
    nd = n_d
    expect = np.stack([1 - 0.999 * nd[:, 0] ** 2, -0.999 * nd[:, 0] * nd[:, 1], -0.999 * nd[:, 0] * nd[:, 2],
                       1 - 0.999 * nd[:, 1] ** 2, -0.999 * nd[:, 1] * nd[:, 2], 1 - 0.999 * nd[:, 2] ** 2], 1)
    assert np.allclose(creg_d, expect, atol=1e-15)
    return int(well.sum()), int((~well).sum())


def compare_full(dev, xyz, r, k, sensor):
    o = pp.preprocess(xyz, r, k, sensor)
    assert dev["xyz"].shape == o["xyz"].shape
    assert np.array_equal(dev["xyz"], o["xyz"])
    assert np.array_equal(dev["counts"], o["counts"])
    assert np.array_equal(dev["nbr"], o["nbr"].astype(np.int32))
    assert np.array_equal(dev["d2"], o["d2"])
    return check_cov_normals(dev, np.arange(len(o["xyz"])), o["xyz"], o["nbr"], sensor)


def test_small_frame_full(vg, frame):
    vgicp, ctx = vg
    pts, sensor = frame
    xyz = pts[::16]
    print("points", len(xyz), flush=True)
    dev = device(vgicp, ctx, xyz, 0.5, 10, sensor)
    well, ill = compare_full(dev, xyz, 0.5, 10, sensor)
    print("downsampled", len(dev["xyz"]), "well-conditioned normals", well, "ill", ill, flush=True)


@pytest.mark.parametrize("k", [1, 7, 16, 32])
def test_neighbour_counts(vg, frame, k):
    vgicp, ctx = vg
    pts, sensor = frame
    xyz = pts[::32]
    dev = device(vgicp, ctx, xyz, 0.5, k, sensor)
    compare_full(dev, xyz, 0.5, k, sensor)


def test_full_frame_sampled(vg, frame):
    """Full 128-ring frame at 0.25 m: every downsampled point bit-exact, k-NN and
    covariances on 600 sampled points (brute force per query)."""
    vgicp, ctx = vg
    pts, sensor = frame
    r, k = 0.25, 10
    dev = device(vgicp, ctx, pts, r, k, sensor)
    c, keys, cnt = pp.downsample(pts, r)
    print("raw", len(pts), "downsampled", len(c), flush=True)
    assert np.array_equal(dev["xyz"], c)
    assert np.array_equal(dev["counts"], cnt)
    q = np.random.default_rng(0).choice(len(c), 600, replace=False)
    idx, d2 = pp.knn(c, k, queries=q)
    assert np.array_equal(dev["nbr"][q], idx.astype(np.int32))
    assert np.array_equal(dev["d2"][q], d2)
    check_rows({key: dev[key][q] for key in ("cov", "cov_raw", "normals")}, c, q, idx, sensor)


def check_rows(dev_rows, P, q, nbr_o, sensor):
    """Covariance / normal checks on sampled rows q (oracle neighbours nbr_o of those rows)."""
    C = pp.covariance(P, nbr_o)
    Creg, n_o, w = pp.regularize(C, P[q], sensor)
    lam = np.maximum(w[:, 2], 1e-300)
    err = np.abs(dev_rows["cov_raw"] - pp.cov6(C)).max(axis=1)
    assert np.all(err <= 1e-11 * lam + 1e-18), err.max()
    gap = (w[:, 1] - w[:, 0]) / lam
    well = gap > 1e-6
    tol = 1e-11 / np.maximum(gap, 1e-300) + 1e-12
    ray = sensor[None] - P[q]
    marg = np.abs(np.einsum("ni,ni->n", n_o, ray)) / np.maximum(np.linalg.norm(ray, axis=1), 1e-300)
    n_d = dev_rows["normals"]
    sgn = np.where((marg < 1e-9) & (np.einsum("ni,ni->n", n_d, n_o) < 0), -1.0, 1.0)
    dn = np.linalg.norm(n_d - sgn[:, None] * n_o, axis=1)
    assert np.all(dn[well] <= tol[well])
    assert np.all(np.abs(dev_rows["cov"] - pp.cov6(Creg))[well].max(axis=1) <= 2 * tol[well] + 1e-15)


def test_far_negative_coordinates(vg, frame):
    """Keys far from zero and negative: the frame moved by (-5000, 3000, -20) m."""
    vgicp, ctx = vg
    pts, sensor = frame
    shift = np.array([-5000.0, 3000.0, -20.0])
    xyz = pts[::16] + shift
    dev = device(vgicp, ctx, xyz, 0.5, 10, sensor + shift)
    compare_full(dev, xyz, 0.5, 10, sensor + shift)


def test_lattice_ties_by_index(vg):
    """One point per voxel at the voxel centre: many exactly equal distances."""
    vgicp, ctx = vg
    g = np.stack(np.meshgrid(np.arange(-6, 6), np.arange(-5, 5), np.arange(0, 3), indexing="ij"), -1)
    xyz = (g.reshape(-1, 3) + 0.5) * 0.5
    xyz = xyz[np.random.default_rng(1).permutation(len(xyz))]
    dev = device(vgicp, ctx, xyz, 0.5, 12, np.array([0.3, 0.2, 9.0]))
    compare_full(dev, xyz, 0.5, 12, np.array([0.3, 0.2, 9.0]))


def test_edge_cases(vg):
    vgicp, ctx = vg
    s = np.zeros(3)
    assert device(vgicp, ctx, np.zeros((0, 3)), 0.5, 10, s)["xyz"].shape == (0, 3)
    one = device(vgicp, ctx, np.array([[1.25, -2.5, 0.75]]), 0.5, 10, s)
    assert np.array_equal(one["xyz"], [[1.25, -2.5, 0.75]])
    assert np.array_equal(one["nbr"][0], [0] + [-1] * 9)
    assert np.all(one["cov_raw"] == 0) and np.isclose(np.linalg.norm(one["normals"][0]), 1.0)
    # every point in one voxel
    rng = np.random.default_rng(2)
    blob = rng.uniform(0.01, 0.99, size=(300, 3)) + [3.0, 4.0, 5.0]
    d = device(vgicp, ctx, blob, 1.0, 5, s)
    compare_full(d, blob, 1.0, 5, s)
    assert len(d["xyz"]) == 1 and d["counts"][0] == 300
    # duplicated points across many voxels: duplicates merge into their voxel's mean
    dup = np.repeat(rng.uniform(-3, 3, size=(200, 3)), 3, axis=0)
    compare_full(device(vgicp, ctx, dup, 0.25, 8, s), dup, 0.25, 8, s)
    # two far-apart clusters (the search reaches the cube bound or scans every point)
    far = np.concatenate([rng.uniform(0, 1, size=(6, 3)), rng.uniform(0, 1, size=(6, 3)) + [400.0, 0, 0]])
    compare_full(device(vgicp, ctx, far, 0.05, 10, s), far, 0.05, 10, s)


def test_isolated_cluster_near_dense_surfaces(vg):
    """A 5-point cluster 10 m from dense walls: its 10 nearest neighbours need a
    search radius of ~10 m through thousands of wall points, which the grid walk
    hands over to the wave-wide pass."""
    vgicp, ctx = vg
    rng = np.random.default_rng(3)
    u = rng.uniform(-15, 15, size=(40000, 2))
    walls = np.concatenate([np.stack([u[:20000, 0], np.full(20000, 10.0), rng.uniform(0, 3, 20000)], 1),
                            np.stack([np.full(20000, -10.0), u[20000:, 1], rng.uniform(0, 3, 20000)], 1)])
    cluster = np.array([0.0, 0.0, 1.5]) + rng.uniform(-0.3, 0.3, size=(5, 3))
    xyz = np.concatenate([walls, cluster])
    sensor = np.array([0.0, 0.0, 1.0])
    dev = device(vgicp, ctx, xyz, 0.1, 10, sensor)
    c, _, _ = pp.downsample(xyz, 0.1)
    assert np.array_equal(dev["xyz"], c)
    far = np.nonzero(np.linalg.norm(c - [0.0, 0.0, 1.5], axis=1) < 1.0)[0]
    q = np.concatenate([far, np.random.default_rng(0).choice(len(c), 200, replace=False)])
    idx, d2 = pp.knn(c, 10, queries=q)
    assert np.array_equal(dev["nbr"][q], idx.astype(np.int32))
    assert np.array_equal(dev["d2"][q], d2)
    check_rows({key: dev[key][q] for key in ("cov", "cov_raw", "normals")}, c, q, idx, sensor)


def test_invalid_arguments(vg):
    vgicp, ctx = vg
    from paper_2407_10344_amd._lib import VGError
    xyz = np.zeros((4, 3))
    for r, k in [(0.0, 10), (-1.0, 10), (np.nan, 10), (0.5, 0), (0.5, 33)]:
        with pytest.raises(VGError) as ei:
            vgicp.Cloud(ctx, xyz, r, k, np.zeros(3))
        assert ei.value.status == -1
    bad = xyz.copy()
    bad[1, 2] = np.inf
    with pytest.raises(VGError) as ei:
        vgicp.Cloud(ctx, bad, 0.5, 10, np.zeros(3))
    assert ei.value.status == -1
    with pytest.raises(VGError) as ei:
        vgicp.Cloud(ctx, np.array([[1e6, 0.0, 0.0]]), 0.25, 10, np.zeros(3))
    assert ei.value.status == -4


@pytest.mark.parametrize("validate", [False, True])
def test_preprocessed_clouds_feed_the_factor(vg, frame, validate):
    """Two halves of a frame, preprocessed on the device, matched by one factor in
    FP64 mode; the oracle preprocesses the same raw halves itself."""
    vgicp, ctx = vg
    pts, sensor = frame
    T0 = synth.random_pose(np.random.default_rng(5), 2.0, 0.2)
    tgt_raw = pts[0::2]
    src_raw = (pts[1::2] - T0[:3, 3]) @ T0[:3, :3]     # source frame = T0^-1 (target frame)
    src_sensor = (sensor - T0[:3, 3]) @ T0[:3, :3]
    res = [0.5, 1.0]
    cs = vgicp.Cloud(ctx, src_raw, 0.25, 10, src_sensor)
    ct = vgicp.Cloud(ctx, tgt_raw, 0.25, 10, sensor)
    src = vgicp.Source.from_cloud(ctx, cs)
    vm = vgicp.VoxelMap.from_cloud(ctx, ct, res)
    cs.close()
    ct.close()
    batch = vgicp.FactorBatch(ctx, [src], [vm], viewpoints=np.array([sensor]), precision="fp64",
                              validation=validate, use_graph=True)
    os_ = pp.preprocess(src_raw, 0.25, 10, src_sensor)
    ot = pp.preprocess(tgt_raw, 0.25, 10, sensor)
    omap = oracle.VoxelMap(ot["xyz"], pp.cov6(ot["cov"]), res)
    ofac = oracle.Factor(os_["xyz"], pp.cov6(os_["cov"]), omap, nrm=os_["normals"], viewpoint=sensor,
                         validate=validate)
    for pose in (T0 @ synth.random_pose(np.random.default_rng(6), 1.0, 0.1), T0):
        e, H, b, inl = batch.linearize(np.array([pose]))
        errs, stats = check_factor(batch, 0, pose, ofac, e[0], H[0], b[0], rel=1e-8)
        print("validate", validate, "errors", errs, "inliers", inl[0].tolist(), flush=True)
    batch.close()
    src.close()
    vm.close()
