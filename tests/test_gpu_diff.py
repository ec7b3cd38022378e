"""Backward kernel and torch.autograd.Function against the FP64 oracle (needs an MI355X).

The oracle gradient (exact, W recomputed, correspondences held) is itself
pinned to central finite differences in the CPU suite.  Here the device
gradient must match it within relative 1e-5 (FP32-compensated) for the pose
tangent and the per-point gradients, and the SE(3) retraction and right
Jacobian used by the autograd Function are checked against scipy's matrix
exponential.
"""

import math

import numpy as np
import pytest
import torch
from scipy.linalg import expm, logm

import oracle
from oracle.parity import frozen_from_device_keys
import synth
from oracle.parity import rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    from paper_2407_10344_amd import vgicp
    ctx = vgicp.Context(0)
    yield vgicp, ctx
    ctx.close()


def twist(xi):
    w, v = xi[:3], xi[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    X[:3, 3] = v
    return X


def vee(X):
    return np.array([X[2, 1], X[0, 2], X[1, 0], X[0, 3], X[1, 3], X[2, 3]])


def unambiguous_pose(of, T, band=1e-5, tries=20):
    """A pose near T at which no transformed point lies within `band` of a voxel face
    (decided by the oracle alone), so the correspondences are unique."""
    rng = np.random.default_rng(123)
    for _ in range(tries):
        tr = of.linearize(T, trace=True)
        if not np.any(tr["face"] < band):
            return T
        T = T @ expm(twist(rng.normal(size=6) * 1e-4))
    return T


def test_se3_retract_and_right_jacobian(vg):
    vgicp, ctx = vg
    rng = np.random.default_rng(0)
    F = 8
    T0 = np.stack([expm(twist(rng.normal(size=6) * 0.5)) for _ in range(F)])
    scale = np.array([0.0, 1e-6, 1e-3, 1e-2, 0.3, 1.0, 2.0, 2.5])
    xi = rng.normal(size=(F, 6)) * scale[:, None]
    d_T0 = torch.tensor(vgicp.poses12(T0), device="cuda")
    d_xi = torch.tensor(xi, device="cuda")
    T, jr = ctx.se3_retract(d_T0, d_xi)
    T = vgicp.pose4x4(T.cpu().numpy())
    jr = jr.cpu().numpy()
    h = 1e-6
    for f in range(F):
        np.testing.assert_allclose(T[f], T0[f] @ expm(twist(xi[f])), atol=1e-12)
        E = expm(twist(xi[f]))
        Einv = np.linalg.inv(E)
        J = np.zeros((6, 6))
        for j in range(6):
            dp = xi[f].copy()
            dm = xi[f].copy()
            dp[j] += h
            dm[j] -= h
            J[:, j] = (vee(np.real(logm(Einv @ expm(twist(dp))))) - vee(np.real(logm(Einv @ expm(twist(dm)))))) / (2 * h)
        np.testing.assert_allclose(jr[f], J, atol=2e-7)


@pytest.fixture(scope="module")
def diff_case():
    cfg = synth.config1(seed=(4, 0), n_target=30000, n_source=20000)
    of = oracle.factor_from_clouds(cfg["sources"][0], cfg["targets"][0], cfg["resolutions"])
    T = unambiguous_pose(of, cfg["poses_true"][0] @ expm(twist(np.array([0.002, -0.003, 0.001, 0.02, 0.01, -0.01]))))
    return cfg, of, T


def test_backward_matches_oracle_gradient(vg, diff_case):
    vgicp, ctx = vg
    cfg, of, T = diff_case
    maps, srcs, batch = vgicp.build_workload(ctx, cfg)
    d_T = torch.tensor(vgicp.poses12([T]), device="cuda")
    ge = torch.tensor([1.7], dtype=torch.float64, device="cuda")
    gxi, gp = batch.backward_async(d_T, ge, points_dtype=torch.float32)
    torch.cuda.synchronize()
    g_o, gm_o = of.gradient(T)
    e_xi = rel_err(gxi.cpu().numpy()[0], 1.7 * g_o)
    e_pt = rel_err(gp.cpu().numpy().astype(np.float64), 1.7 * gm_o)
    print("backward rel err: xi %.3g points %.3g" % (e_xi, e_pt), flush=True)
    assert e_xi <= 1e-5 and e_pt <= 1e-5
    batch.close()


def test_autograd_function(vg, diff_case):
    vgicp, ctx = vg
    from paper_2407_10344_amd.autograd import VGICPCost
    cfg, of, T = diff_case
    maps, srcs, batch = vgicp.build_workload(ctx, cfg)
    src = cfg["sources"][0]
    pts = torch.tensor(src.xyz64(), dtype=torch.float32, device="cuda", requires_grad=True)
    xi = torch.zeros((1, 6), dtype=torch.float64, device="cuda", requires_grad=True)
    T0 = torch.tensor(vgicp.poses12([T]), device="cuda")
    e = VGICPCost.apply(xi, pts, batch, T0)
    (3.0 * e.sum()).backward()
    torch.cuda.synchronize()
    assert rel_err(e.detach().cpu().numpy()[0], of.evaluate(T)) <= 1e-5
    g_o, gm_o = of.gradient(T)
    assert rel_err(xi.grad.cpu().numpy()[0], 3.0 * g_o) <= 1e-5
    assert rel_err(pts.grad.cpu().numpy().astype(np.float64), 3.0 * gm_o) <= 1e-5
    batch.close()


def test_autograd_fd_fp64_nonzero_tangent(vg):
    """FP64 device path, xi != 0: autograd gradient == central FD of the device forward.

    One-point-per-voxel lattice clouds with offsets 0.1 m from every face keep the
    correspondences fixed under the 1e-6 perturbations of the difference quotient.
    """
    vgicp, ctx = vg
    from paper_2407_10344_amd.autograd import VGICPCost
    cloud, res = synth.tiny_lattice_pair(3, resolutions=(1.0,))
    rng = np.random.default_rng(5)
    moved = cloud.xyz64() + rng.normal(scale=0.02, size=(cloud.n, 3))
    m = vgicp.VoxelMap(ctx, cloud.xyz64(), cloud.cov64(), res)
    src = vgicp.Source(ctx, moved, cloud.cov64())
    batch = vgicp.FactorBatch(ctx, [src], [m], precision="fp64")
    T0 = torch.tensor(vgicp.poses12([expm(twist(np.array([0.01, 0, 0, 0, 0.01, 0])))]), device="cuda")
    xi0 = np.array([[0.003, -0.002, 0.004, 0.01, -0.02, 0.005]])
    pts = torch.tensor(moved, device="cuda", requires_grad=True)
    xi = torch.tensor(xi0, device="cuda", requires_grad=True)
    e = VGICPCost.apply(xi, pts, batch, T0)
    e.sum().backward()
    g = xi.grad.cpu().numpy()[0]
    gp = pts.grad.cpu().numpy()
    h = 1e-6
    fd = np.zeros(6)
    with torch.no_grad():
        for j in range(6):
            xp = xi0.copy()
            xm = xi0.copy()
            xp[0, j] += h
            xm[0, j] -= h
            ep = VGICPCost.apply(torch.tensor(xp, device="cuda"), pts.detach(), batch, T0).item()
            em = VGICPCost.apply(torch.tensor(xm, device="cuda"), pts.detach(), batch, T0).item()
            fd[j] = (ep - em) / (2 * h)
        k = 7
        fdp = np.zeros(3)
        for a in range(3):
            P = pts.detach().clone()
            P[k, a] += h
            ep = VGICPCost.apply(torch.tensor(xi0, device="cuda"), P, batch, T0).item()
            P[k, a] -= 2 * h
            em = VGICPCost.apply(torch.tensor(xi0, device="cuda"), P, batch, T0).item()
            fdp[a] = (ep - em) / (2 * h)
    assert rel_err(g, fd) <= 1e-6, (g, fd)
    assert rel_err(gp[k], fdp) <= 1e-6, (gp[k], fdp)
    batch.close()
    src.close()
    m.close()


@pytest.mark.slow
def test_differentiation_batch_full_size(vg):
    """64 factors x 100k source points; sampled factors against the oracle gradient."""
    vgicp, ctx = vg
    cfg = synth.config4()
    maps, srcs, batch = vgicp.build_workload(ctx, cfg)
    F = len(cfg["factors"])
    poses = np.array(cfg["poses_true"])
    d_T = torch.tensor(vgicp.poses12(poses), device="cuda")
    ge = torch.ones(F, dtype=torch.float64, device="cuda")
    gxi, gp = batch.backward_async(d_T, ge, points_dtype=torch.float32)
    torch.cuda.synchronize()
    gxi = gxi.cpu().numpy()
    gp = gp.cpu().numpy()
    for f in (0, 31, 63):
        s, t = cfg["factors"][f]
        of = oracle.factor_from_clouds(cfg["sources"][s], cfg["targets"][t], cfg["resolutions"])
        # points within 1e-5 m of a voxel face may take either voxel: the oracle
        # gradient is taken on the device's correspondences (frozen), W recomputed
        keys_d, found_d = batch.correspondences(poses[f], f)
        fz, n_face = frozen_from_device_keys(of, poses[f], keys_d, found_d)
        g_o, gm_o = of.gradient(poses[f], frozen=fz)
        row0, n = batch.source_rows[id(srcs[s])]
        ex, ep = rel_err(gxi[f], g_o), rel_err(gp[row0:row0 + n].astype(np.float64), gm_o)
        print("factor", f, "near-face choices", n_face, "rel err xi %.3g points %.3g" % (ex, ep), flush=True)
        assert ex <= 1e-5 and ep <= 1e-5
    batch.close()
