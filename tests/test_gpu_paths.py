"""Option paths and batch-level guarantees through the C ABI (needs an MI355X).

* lane-level Kahan sums (``lane_kahan``) against the FP64 oracle;
* the work counts the kernels report (walked points and chunks, table lookups)
  against what they must be: every point walked where nothing is culled,
  inliers <= lookups <= walked points x levels, identical counts for
  linearize / evaluate / overlap, fewer walked points once chunks are culled;
* point gradients of a source shared by several factors: the sum of the
  oracle's per-factor gradients, bit-identical from one call to the next;
* evaluate's e equal to linearize's e bit for bit in the compensated mode;
* the compensated mode's extent limit (a source spanning kilometres is refused);
* FP32-compensated central differences at h = 1e-4 within their rounding bound.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.parity import REL, check_factor, frozen_from_device_keys, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    from paper_2407_10344_amd import vgicp
    ctx = vgicp.Context(0)
    yield vgicp, ctx
    ctx.close()


@pytest.fixture(scope="module")
def c1():
    return synth.config1(seed=1)


@pytest.fixture(scope="module")
def c2():
    return synth.config2(seed=2)


def oracle_factor(cfg, f, validate=False):
    s, t = cfg["factors"][f]
    return oracle.factor_from_clouds(cfg["sources"][s], cfg["targets"][t], cfg["resolutions"],
                                     viewpoint=cfg["target_viewpoints"][f], validate=validate)


# ----------------------------------------------------------------- lane-level Kahan sums

def test_lane_kahan_single_factor(vg, c1):
    vgicp, ctx = vg
    maps, srcs, batch = vgicp.build_workload(ctx, c1, lane_kahan=True)
    _, _, plain = vgicp.build_workload(ctx, c1)
    of = oracle_factor(c1, 0)
    for pose in (c1["poses"][0], c1["poses_true"][0]):
        e, H, b, inl = batch.linearize([pose])
        errs, stats = check_factor(batch, 0, pose, of, e[0], H[0], b[0])
        print("lane_kahan config1", {k: "%.2g" % v for k, v in errs.items()}, flush=True)
        # same keys and inliers as the uncompensated lanes
        _, _, _, inl2 = plain.linearize([pose])
        assert np.array_equal(inl, inl2)
    plain.close()
    batch.close()


def test_lane_kahan_odometry_batch(vg, c2):
    vgicp, ctx = vg
    maps, srcs, batch = vgicp.build_workload(ctx, c2, lane_kahan=True)
    poses = np.array(c2["poses"])
    e, H, b, inl = batch.linearize(poses)
    worst = {}
    for f in range(len(poses)):
        errs, _ = check_factor(batch, f, poses[f], oracle_factor(c2, f), e[f], H[f], b[f])
        worst = {k: max(worst.get(k, 0.0), v) for k, v in errs.items()}
    print("lane_kahan config2 worst", {k: "%.2g" % v for k, v in worst.items()}, flush=True)
    e2, H2, b2, _ = batch.linearize(poses)
    assert np.array_equal(e, e2) and np.array_equal(H, H2) and np.array_equal(b, b2)
    batch.close()


# ----------------------------------------------------------------- work counts

@pytest.mark.parametrize("prec", ["fp32c", "fp32", "fp64"])
def test_work_counts(vg, c2, prec):
    vgicp, ctx = vg
    maps, srcs, batch = vgicp.build_workload(ctx, c2, precision=prec)
    poses = np.array(c2["poses"])
    n = np.array([c2["sources"][s].n for (s, _) in c2["factors"]])
    _, _, _, inl = batch.linearize(poses)
    wp, wc, lk = batch.work()
    print(prec, "walked", wp[:3].tolist(), "of", n[:3].tolist(), "lookups", lk[0].tolist(), "inliers",
          inl[0].tolist(), flush=True)
    L = batch.L
    assert np.all(wp <= n) and np.all(wc <= (n + 63) // 64)
    assert np.all(inl <= lk) and np.all(lk <= wp[:, None])
    if prec == "fp32":
        # the naive mode culls nothing: every point and chunk is walked
        assert np.array_equal(wp, n) and np.array_equal(wc, (n + 63) // 64)
    # the evaluation and overlap launches probe exactly the same point levels
    batch.evaluate(poses)
    wp2, wc2, lk2 = batch.work()
    assert np.array_equal(wp2, wp) and np.array_equal(wc2, wc) and np.array_equal(lk2, lk)
    ov = batch.overlap(poses)
    wp3, wc3, lk3 = batch.work()
    assert np.array_equal(wp3, wp) and np.array_equal(lk3, lk)
    assert np.array_equal(np.rint(ov * n[:, None]).astype(np.int64), inl)
    batch.close()


def test_work_counts_follow_culling(vg, c1):
    """A source moved half off the target walks fewer points than it has."""
    vgicp, ctx = vg
    src0, tgt, res = c1["sources"][0], c1["targets"][0], c1["resolutions"]
    src = synth.Cloud(origin=src0.origin + np.array([32.0, 0.0, 0.0]), off32=src0.off32, cov32=src0.cov32,
                      nrm32=src0.nrm32, viewpoint=src0.viewpoint)
    m = vgicp.VoxelMap(ctx, tgt.xyz64(), tgt.cov64(), list(res))
    s = vgicp.Source(ctx, src.xyz64(), src.cov64(), src.nrm64())
    pose = c1["poses_true"][0]
    out = {}
    for prec in ("fp32c", "fp64", "fp32"):
        batch = vgicp.FactorBatch(ctx, [s], [m], precision=prec)
        _, _, _, inl = batch.linearize([pose])
        wp, wc, lk = batch.work()
        out[prec] = (int(wp[0]), int(inl[0, 0]))
        assert inl[0, 0] <= lk[0, 0] <= wp[0]
        batch.close()
    print("walked / inliers per mode", out, "of", src.n, flush=True)
    assert out["fp32"][0] == src.n
    assert out["fp32c"][0] < src.n and out["fp64"][0] < src.n
    assert out["fp32c"][1] > 0
    s.close()
    m.close()


# ----------------------------------------------------------------- shared-source backward

@pytest.mark.parametrize("levels", [4, 1])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_shared_source_backward_is_sum_of_oracle_gradients(vg, c2, dtype, levels):
    """The odometry batch matches one new frame against 20 keyframes: every
    factor shares the same source, so its point gradient is the sum of the 20
    factors' gradients (weighted by grad_e), formed in factor order.  With the
    maps cut to their 0.5 m level the one-level backward kernel runs, which
    skips culled chunks and writes only the rows of points with a voxel."""
    vgicp, ctx = vg
    if levels == 1:
        c2 = dict(c2, resolutions=(0.5,))
    maps, srcs, batch = vgicp.build_workload(ctx, c2)
    poses = np.array(c2["poses"])
    F = len(poses)
    assert batch.grad_rows == c2["sources"][0].n     # one distinct source
    d_T = torch.tensor(vgicp.poses12(poses), device="cuda")
    w = np.linspace(0.5, 2.0, F)
    ge = torch.tensor(w, dtype=torch.float64, device="cuda")
    gxi, gp = batch.backward_async(d_T, ge, points_dtype=dtype)
    gxi2, gp2 = batch.backward_async(d_T, ge, points_dtype=dtype)
    torch.cuda.synchronize()
    gxi, gp, gxi2, gp2 = (x.cpu().numpy() for x in (gxi, gp, gxi2, gp2))
    assert np.array_equal(gp, gp2) and np.array_equal(gxi, gxi2)   # deterministic
    want = np.zeros((batch.grad_rows, 3))
    for f in range(F):
        of = oracle_factor(c2, f)
        keys_d, found_d = batch.correspondences(poses[f], f)
        fz, _ = frozen_from_device_keys(of, poses[f], keys_d, found_d)
        g_o, gm_o = of.gradient(poses[f], frozen=fz)
        assert rel_err(gxi[f], w[f] * g_o) <= REL
        want += w[f] * gm_o
    err = rel_err(gp.astype(np.float64), want)
    print("shared source", dtype, levels, "level(s): point gradient rel err %.3g" % err, flush=True)
    assert err <= REL
    batch.close()


# ----------------------------------------------------------------- evaluate and linearize agree

@pytest.mark.parametrize("levels", [4, 1])
def test_evaluate_e_equals_linearize_e(vg, c2, levels):
    """In the compensated mode evaluate and linearize queue the same hits, process
    them in the same lanes with the same operations for e and sum e the same
    way, so evaluate's e at a pose is linearize's e at that pose bit for bit (a
    Levenberg-Marquardt step accepts a candidate by comparing the two)."""
    vgicp, ctx = vg
    cfg = c2 if levels == 4 else dict(c2, resolutions=(0.5,))
    maps, srcs, batch = vgicp.build_workload(ctx, cfg)
    for poses in (np.array(cfg["poses"]), np.array(cfg["poses_true"])):
        e, H, b, inl = batch.linearize(poses)
        e_eval = np.asarray(batch.evaluate(poses))
        print(levels, "level(s): max |e_eval - e_lin| / e = %.3g" % float(np.max(np.abs(e_eval - e) / e)), flush=True)
        assert np.array_equal(e_eval, e)
    batch.close()


# ----------------------------------------------------------------- compensated extent limit

def test_compensated_mode_refuses_kilometre_sources(vg):
    from paper_2407_10344_amd._lib import VGError
    vgicp, ctx = vg
    rng = np.random.default_rng(4)
    n = 4000
    x = np.stack([rng.uniform(0.0, 4000.0, n), rng.uniform(-2.0, 2.0, n), rng.normal(scale=0.05, size=n)], 1)
    cov = np.tile([0.05, 0.0, 0.0, 0.05, 0.0, 0.001], (n, 1))
    m = vgicp.VoxelMap(ctx, x[:200], cov[:200], [0.5])
    s = vgicp.Source(ctx, x, cov)
    with pytest.raises(VGError, match="INVALID_ARG.*VG_FP64"):
        vgicp.FactorBatch(ctx, [s], [m], precision="fp32c")
    ok = vgicp.FactorBatch(ctx, [s], [m], precision="fp64")      # the FP64 mode takes it
    ok.close()
    small = vgicp.Source(ctx, x[x[:, 0] < 300.0], cov[x[:, 0] < 300.0])
    ok = vgicp.FactorBatch(ctx, [small], [m], precision="fp32c")  # within the limit
    ok.close()
    for o in (s, small, m):
        o.close()


# ----------------------------------------------------------------- FP32 central differences

def test_fd_fp32c_h1e4_within_rounding_bound(vg):
    """Central differences of the compensated-FP32 device error at h = 1e-4 match
    the device gradient within the FD error bound: rounding 2 eps |e| / (2 h)
    (eps = relative error of one evaluation) plus the O(h^2) truncation term,
    on one-point-per-voxel lattice clouds whose correspondences cannot change
    under the perturbation (offsets 0.1 m from every face)."""
    vgicp, ctx = vg
    from paper_2407_10344_amd.autograd import VGICPCost
    cloud, res = synth.tiny_lattice_pair(7, resolutions=(1.0,))
    rng = np.random.default_rng(9)
    moved = cloud.xyz64() + rng.normal(scale=0.02, size=(cloud.n, 3))
    m = vgicp.VoxelMap(ctx, cloud.xyz64(), cloud.cov64(), res)
    src = vgicp.Source(ctx, moved, cloud.cov64())
    batch = vgicp.FactorBatch(ctx, [src], [m], precision="fp32c")
    T0 = torch.tensor(vgicp.poses12([np.eye(4)]), device="cuda")
    pts = torch.tensor(moved, device="cuda")
    xi = torch.zeros((1, 6), dtype=torch.float64, device="cuda", requires_grad=True)
    e = VGICPCost.apply(xi, pts, batch, T0)
    e.sum().backward()
    g = xi.grad.cpu().numpy()[0]
    e0 = float(e.item())
    of = oracle.Factor(moved, cloud.cov64(), oracle.VoxelMap(cloud.xyz64(), cloud.cov64(), res))
    eps = 1e-6   # bound of the device error's relative deviation from the FP64 oracle (measured below)
    assert rel_err(e0, of.evaluate(np.eye(4))) < eps
    h = 1e-4
    fd = np.zeros(6)
    with torch.no_grad():
        for j in range(6):
            xp = np.zeros((1, 6))
            xm = np.zeros((1, 6))
            xp[0, j] = h
            xm[0, j] = -h
            ep = VGICPCost.apply(torch.tensor(xp, device="cuda"), pts, batch, T0).item()
            em = VGICPCost.apply(torch.tensor(xm, device="cuda"), pts, batch, T0).item()
            fd[j] = (ep - em) / (2 * h)
    # truncation: |e'''| h^2 / 6, with e''' bounded by the oracle's FD of the exact gradient
    g_o, _ = of.gradient(np.eye(4))
    bound = 2 * eps * abs(e0) / (2 * h) + 1e-3 * np.linalg.norm(g_o) + 1e-12
    print("fd fp32c h=1e-4: |fd - g| max %.3g, bound %.3g, |g| %.3g" % (np.max(np.abs(fd - g)), bound,
                                                                     np.linalg.norm(g)), flush=True)
    assert np.max(np.abs(fd - g)) <= bound
    assert rel_err(g, g_o) <= REL
    batch.close()
    src.close()
    m.close()
