"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test fixes part of the oracle with something independent of it: values
worked out by hand (tests/golden), brute-force search, invariances of the
cost, finite differences of its own error (through scipy's matrix exponential,
not the oracle's), and a special case that reduces to the Kabsch/Umeyama SVD.
A plausible slip (dropped term, wrong sign, transposed operand, floor vs
truncation, wrong perturbation side) fails at least one of them.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def twist(xi):
    """4x4 matrix of xi = [omega; v] in se(3)."""
    w, v = xi[:3], xi[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    X[:3, 3] = v
    return X


def retract(T, xi):
    return T @ expm(twist(np.asarray(xi, dtype=np.float64)))


def adjoint(T):
    """Ad_T acting on xi = [omega; v]."""
    Rm, t = T[:3, :3], T[:3, 3]
    tx = np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])
    A = np.zeros((6, 6))
    A[:3, :3] = Rm
    A[3:, 3:] = Rm
    A[3:, :3] = tx @ Rm
    return A


def rigid(rng, deg, m):
    T = np.eye(4)
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    T[:3, :3] = Rotation.from_rotvec(ax * math.radians(deg)).as_matrix()
    d = rng.normal(size=3)
    T[:3, 3] = d / np.linalg.norm(d) * m
    return T


def cov6_rotate(cov6, Rm):
    C = np.stack([cov6[:, [0, 1, 2]], cov6[:, [1, 3, 4]], cov6[:, [2, 4, 5]]], axis=1)
    C2 = Rm[None] @ C @ Rm.T[None]
    return np.stack([C2[:, 0, 0], C2[:, 0, 1], C2[:, 0, 2], C2[:, 1, 1], C2[:, 1, 2], C2[:, 2, 2]], axis=1)


@pytest.fixture(scope="module")
def c1_small():
    cfg = synth.config1(seed=101, n_target=6000, n_source=1500)
    f = oracle.factor_from_clouds(cfg["sources"][0], cfg["targets"][0], cfg["resolutions"])
    return cfg, f


# ---------------------------------------------------------------- golden / closed forms

@pytest.mark.parametrize("name", ["single_point_isotropic.json", "single_point_diagonal.json"])
def test_single_point_by_hand(name):
    g = json.load(open(os.path.join(GOLD, name)))
    vm = oracle.VoxelMap(np.array(g["target_xyz"]), np.array(g["target_cov"]), [g["resolution"]])
    f = oracle.Factor(np.array(g["source_xyz"]), np.array(g["source_cov"]), vm)
    r = f.linearize(np.array(g["pose"], dtype=np.float64))
    assert r["inliers"].tolist() == [1]
    assert r["e"] == pytest.approx(g["e"], abs=1e-14)
    np.testing.assert_allclose(r["b"], g["b"], atol=1e-14)
    np.testing.assert_allclose(r["H"], np.array(g["H"]), atol=1e-14)


def test_voxel_stats_by_hand():
    g = json.load(open(os.path.join(GOLD, "voxel_stats_by_hand.json")))
    k, m, c, n = oracle.voxelize(np.array(g["xyz"]), np.array(g["cov"]), g["resolution"])
    assert k.tolist() == g["keys"]
    assert n.tolist() == g["counts"]
    np.testing.assert_allclose(m, g["means"], atol=1e-15)
    np.testing.assert_allclose(c, g["covs"], atol=1e-15)


# ---------------------------------------------------------------- voxelization, brute force

def test_voxelize_brute_force_containment():
    rng = np.random.default_rng(5)
    xyz = rng.uniform(-1.3, 1.3, (300, 3))
    cov = rng.uniform(0.1, 1.0, (300, 6))
    for r in (0.25, 0.5, 1.0):
        keys, means, covs, counts = oracle.voxelize(xyz, cov, r)
        # keys strictly ascending lexicographically
        assert all(tuple(keys[i]) < tuple(keys[i + 1]) for i in range(len(keys) - 1))
        assigned = np.zeros(xyz.shape[0], dtype=int)
        for v in range(keys.shape[0]):
            lo = keys[v] * r
            hi = (keys[v] + 1) * r
            inside = np.all((xyz >= lo) & (xyz < hi), axis=1)     # the voxel's box, by comparison
            assert inside.sum() == counts[v]
            assigned += inside
            np.testing.assert_allclose(means[v], xyz[inside].mean(axis=0), rtol=0, atol=1e-15)
            np.testing.assert_allclose(covs[v], cov[inside].mean(axis=0), rtol=0, atol=1e-15)
        assert np.all(assigned == 1)


def test_lookup_brute_force(c1_small):
    """Each inlier's voxel is the unique voxel whose box contains y (scan of every voxel)."""
    cfg, f = c1_small
    T = retract(np.eye(4), [0.01, -0.02, 0.015, 0.05, -0.03, 0.02])
    tr = f.linearize(T, trace=True)
    keys, _, _, _ = f.vmap.levels[0]
    r = f.vmap.resolutions[0]
    lo = keys * r
    hi = (keys + 1) * r
    y = f.xyz @ T[:3, :3].T + T[:3, 3]
    sel = np.random.default_rng(0).choice(f.n, 400, replace=False)
    for k in sel:
        inside = np.nonzero(np.all((y[k] >= lo) & (y[k] < hi), axis=1))[0]
        v = tr["vidx"][k, 0]
        if inside.size == 0:
            assert v == -1
        else:
            assert inside.size == 1 and v == inside[0]


def test_negative_coordinates_floor_not_truncate():
    xyz = np.array([[-0.01, -0.01, -0.01], [0.01, 0.01, 0.01]])
    cov = np.tile([1.0, 0, 0, 1, 0, 1], (2, 1))
    k, _, _, n = oracle.voxelize(xyz, cov, 0.5)
    assert k.tolist() == [[-1, -1, -1], [0, 0, 0]]


# ---------------------------------------------------------------- zero residual and PSD

def test_zero_residual_lattice():
    cloud, res = synth.tiny_lattice_pair(0)
    vm = oracle.VoxelMap(cloud.xyz64(), cloud.cov64(), res)
    f = oracle.Factor(cloud.xyz64(), cloud.cov64(), vm)
    r = f.linearize(np.eye(4))
    assert r["e"] == 0.0
    assert np.all(r["b"] == 0.0)
    assert r["inliers"].tolist() == [cloud.n] * len(res)
    w = np.linalg.eigvalsh(r["H"])
    assert w.min() > 0


def test_H_symmetric_psd(c1_small):
    cfg, f = c1_small
    for T in (np.eye(4), cfg["poses_true"][0]):
        r = f.linearize(T)
        H = r["H"]
        np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-13 * np.abs(H).max())
        w = np.linalg.eigvalsh(H)
        assert w.min() >= -1e-12 * np.abs(w).max()


# ---------------------------------------------------------------- derivatives

def _frozen(f, T):
    return f.linearize(T, trace=True)["vidx"]


def test_b_is_half_gradient_of_frozen_gn_cost(c1_small):
    """b = 1/2 d/dxi [sum d(xi)^T W0 d(xi)] with W and correspondences frozen (central FD)."""
    cfg, f = c1_small
    T0 = cfg["poses_true"][0] @ rigid(np.random.default_rng(1), 0.5, 0.05)
    fz = _frozen(f, T0)
    r = f.linearize(T0)
    h = 1e-5
    g = np.zeros(6)
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        ep = f.evaluate(retract(T0, e), frozen=fz, omega_pose=T0)
        em = f.evaluate(retract(T0, -e), frozen=fz, omega_pose=T0)
        g[j] = (ep - em) / (2 * h)
    np.testing.assert_allclose(r["b"], g / 2, rtol=1e-6, atol=1e-6 * np.abs(g).max())


def test_H_is_half_hessian_at_zero_residual():
    """At d = 0 the Omega-derivative terms vanish: H = 1/2 Hessian of e (FD, Omega recomputed)."""
    cloud, res = synth.tiny_lattice_pair(1, resolutions=(0.5, 1.0))
    vm = oracle.VoxelMap(cloud.xyz64(), cloud.cov64(), res)
    f = oracle.Factor(cloud.xyz64(), cloud.cov64(), vm)
    T0 = np.eye(4)
    fz = _frozen(f, T0)
    H = f.linearize(T0)["H"]
    h = 1e-4
    Hfd = np.zeros((6, 6))
    E = np.eye(6) * h
    for i in range(6):
        for j in range(6):
            epp = f.evaluate(retract(T0, E[i] + E[j]), frozen=fz)
            epm = f.evaluate(retract(T0, E[i] - E[j]), frozen=fz)
            emp = f.evaluate(retract(T0, -E[i] + E[j]), frozen=fz)
            emm = f.evaluate(retract(T0, -E[i] - E[j]), frozen=fz)
            Hfd[i, j] = (epp - epm - emp + emm) / (4 * h * h)
    np.testing.assert_allclose(H, Hfd / 2, rtol=1e-5, atol=1e-5 * np.abs(H).max())


def test_jacobian_per_point_isotropic():
    """With C = C~ = I/2 we get W = I, so e = sum |d|^2 exactly; FD of e fixes b for a single point."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        mu = rng.uniform(0.05, 0.95, (1, 3))
        tgt = rng.uniform(0.05, 0.95, (1, 3))
        iso = np.array([[0.5, 0, 0, 0.5, 0, 0.5]])
        vm = oracle.VoxelMap(tgt, iso, [1.0])
        f = oracle.Factor(mu, iso, vm)
        T0 = np.eye(4)
        fz = _frozen(f, T0)
        r = f.linearize(T0)
        h = 1e-6
        g = np.zeros(6)
        for j in range(6):
            e = np.zeros(6)
            e[j] = h
            g[j] = (f.evaluate(retract(T0, e), frozen=fz) - f.evaluate(retract(T0, -e), frozen=fz)) / (2 * h)
        np.testing.assert_allclose(r["b"], g / 2, atol=1e-8)
        d = tgt[0] - mu[0]
        assert r["e"] == pytest.approx(d @ d, rel=1e-14)


def test_exact_gradient_vs_fd(c1_small):
    """Oracle gradient (Omega recomputed) vs central FD of e with frozen correspondences, h = 1e-4."""
    cfg, f = c1_small
    T0 = cfg["poses_true"][0] @ rigid(np.random.default_rng(2), 1.0, 0.1)
    fz = _frozen(f, T0)
    g, gm = f.gradient(T0)
    h = 1e-4
    gfd = np.zeros(6)
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        gfd[j] = (f.evaluate(retract(T0, e), frozen=fz) - f.evaluate(retract(T0, -e), frozen=fz)) / (2 * h)
    np.testing.assert_allclose(g, gfd, rtol=1e-5, atol=1e-6 * np.abs(gfd).max())
    # de/dv equals the sum of de/dmu_k (a translation of the perturbation moves every point)
    np.testing.assert_allclose(g[3:], gm.sum(axis=0), rtol=1e-10, atol=1e-9 * np.abs(g).max())


def test_point_gradient_vs_fd(c1_small):
    cfg, f = c1_small
    T0 = cfg["poses_true"][0]
    fz = _frozen(f, T0)
    _, gm = f.gradient(T0)
    inl = np.nonzero(fz[:, 0] >= 0)[0][:5]
    h = 1e-5
    for k in inl:
        for a in range(3):
            xyz0 = f.xyz.copy()
            f.xyz[k, a] += h
            ep = f.evaluate(T0, frozen=fz)
            f.xyz[:] = xyz0
            f.xyz[k, a] -= h
            em = f.evaluate(T0, frozen=fz)
            f.xyz[:] = xyz0
            assert gm[k, a] == pytest.approx((ep - em) / (2 * h), rel=1e-5, abs=1e-7)


# ---------------------------------------------------------------- invariances

def test_invariance_rigid_source_change(c1_small):
    """Moving the source cloud by G and the pose by G^-1 leaves e; H, b transform by Ad_{G^-1}."""
    cfg, f = c1_small
    rng = np.random.default_rng(7)
    T = cfg["poses_true"][0] @ rigid(rng, 1.0, 0.1)
    G = rigid(rng, 37.0, 4.0)
    xyz2 = f.xyz @ G[:3, :3].T + G[:3, 3]
    cov2 = cov6_rotate(f.cov, G[:3, :3])
    f2 = oracle.Factor(xyz2, cov2, f.vmap)
    T2 = T @ np.linalg.inv(G)
    r1 = f.linearize(T, trace=True)
    r2 = f2.linearize(T2, trace=True)
    assert np.array_equal(r1["vidx"], r2["vidx"])
    assert r2["e"] == pytest.approx(r1["e"], rel=1e-11)
    A = adjoint(np.linalg.inv(G))
    np.testing.assert_allclose(r2["H"], A.T @ r1["H"] @ A, rtol=1e-9, atol=1e-9 * np.abs(r1["H"]).max())
    np.testing.assert_allclose(r2["b"], A.T @ r1["b"], rtol=1e-9, atol=1e-9 * np.abs(r1["b"]).max())


@pytest.mark.parametrize("perm_seed", [0, 1, 2])
def test_invariance_lattice_preserving_common_transform(c1_small, perm_seed):
    """A transform in the voxel lattice's symmetry group (axis permutation/sign flip with
    determinant +1, translation by whole coarse voxels) applied to both clouds leaves e."""
    cfg, f = c1_small
    rng = np.random.default_rng(perm_seed)
    while True:
        P = np.eye(3)[rng.permutation(3)] * rng.choice([-1, 1], 3)[:, None]
        if np.linalg.det(P) > 0:
            break
    G = np.eye(4)
    G[:3, :3] = P
    G[:3, 3] = rng.integers(-5, 6, 3) * 0.5
    tgt = cfg["targets"][0]
    xyz = tgt.xyz64()
    # a coordinate lying exactly on a face changes voxel under a sign flip (the
    # half-open cell flips side); FP32-rounded inputs can land there, so drop them
    on_face = np.any(xyz / 0.5 == np.floor(xyz / 0.5), axis=1)
    xyz, tc = xyz[~on_face], tgt.cov64()[~on_face]
    vm1 = oracle.VoxelMap(xyz, tc, cfg["resolutions"])
    f = oracle.Factor(f.xyz, f.cov, vm1)
    txyz = xyz @ P.T + G[:3, 3]
    tcov = cov6_rotate(tc, P)
    vm2 = oracle.VoxelMap(txyz, tcov, cfg["resolutions"])
    sxyz = f.xyz @ P.T + G[:3, 3]
    f2 = oracle.Factor(sxyz, cov6_rotate(f.cov, P), vm2)
    T = cfg["poses_true"][0]
    T2 = G @ T @ np.linalg.inv(G)
    r1 = f.linearize(T, trace=True)
    r2 = f2.linearize(T2, trace=True)
    near = (r1["face"] < 1e-9) | (r2["face"] < 1e-9)
    assert not near.any()
    assert np.array_equal(r1["inliers"], r2["inliers"])
    assert r2["e"] == pytest.approx(r1["e"], rel=1e-10)


def test_multilevel_is_sum_of_levels():
    cfg = synth.config1(seed=102, n_target=4000, n_source=1000, resolutions=(0.25, 0.5, 1.0))
    s, t = cfg["sources"][0], cfg["targets"][0]
    T = cfg["poses_true"][0] @ rigid(np.random.default_rng(3), 0.5, 0.05)
    full = oracle.factor_from_clouds(s, t, cfg["resolutions"]).linearize(T)
    e, H, b = 0.0, np.zeros((6, 6)), np.zeros(6)
    for r in cfg["resolutions"]:
        one = oracle.factor_from_clouds(s, t, [r]).linearize(T)
        e += one["e"]
        H += one["H"]
        b += one["b"]
    assert full["e"] == pytest.approx(e, rel=1e-12)
    np.testing.assert_allclose(full["H"], H, rtol=1e-12, atol=1e-12 * np.abs(H).max())
    np.testing.assert_allclose(full["b"], b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


# ---------------------------------------------------------------- special cases

def test_isotropic_gn_fixed_point_is_kabsch():
    """C = C~ = s I makes W constant: Gauss-Newton on frozen pairs must reach the SVD
    (Kabsch/Umeyama) least-squares alignment of the points to their voxel means."""
    rng = np.random.default_rng(11)
    cfg = synth.config1(seed=103, n_target=3000, n_source=800)
    s, t = cfg["sources"][0], cfg["targets"][0]
    iso = np.tile([0.05, 0, 0, 0.05, 0, 0.05], (s.n, 1))
    isot = np.tile([0.05, 0, 0, 0.05, 0, 0.05], (t.n, 1))
    vm = oracle.VoxelMap(t.xyz64(), isot, [0.5])
    f = oracle.Factor(s.xyz64(), iso, vm)
    T0 = cfg["poses_true"][0] @ rigid(rng, 0.3, 0.03)
    tr = f.linearize(T0, trace=True)
    fz = tr["vidx"]
    pairs = fz[:, 0] >= 0
    P = f.xyz[pairs]
    Q = vm.levels[0][1][fz[pairs, 0]]
    # Kabsch: min sum |Q - (R P + t)|^2
    pm, qm = P.mean(0), Q.mean(0)
    U, S, Vt = np.linalg.svd((Q - qm).T @ (P - pm))
    D = np.diag([1, 1, np.sign(np.linalg.det(U @ Vt))])
    Rk = U @ D @ Vt
    tk = qm - Rk @ pm
    T = T0.copy()
    for _ in range(30):
        r = f.linearize(T, frozen=fz)
        delta = -np.linalg.solve(r["H"], r["b"])
        T = retract(T, delta)
    np.testing.assert_allclose(T[:3, :3], Rk, atol=1e-10)
    np.testing.assert_allclose(T[:3, 3], tk, atol=1e-9)


def test_lm_converges_on_lattice():
    """From a small offset on a one-point-per-voxel lattice the LM loop returns to identity."""
    cloud, res = synth.tiny_lattice_pair(2, resolutions=(1.0,))
    vm = oracle.VoxelMap(cloud.xyz64(), cloud.cov64(), res)
    f = oracle.Factor(cloud.xyz64(), cloud.cov64(), vm)
    T0 = rigid(np.random.default_rng(4), 0.2, 0.01)
    out = f.lm(T0, iters=10, lambda0=1e-4)
    assert out["accepted"][0]
    np.testing.assert_allclose(out["pose"], np.eye(4), atol=1e-9)
    assert out["e"][0] > out["e"][-1]


def test_se3_exp_matches_matrix_exponential():
    rng = np.random.default_rng(9)
    for scale in (1e-7, 1e-3, 0.3, 2.0):
        xi = rng.normal(size=6) * scale
        np.testing.assert_allclose(oracle.se3_exp(xi), expm(twist(xi)), atol=1e-13)


def test_visibility_rule():
    """Discard when (mu - T^-1 c) . n > 0, keep otherwise (ties kept)."""
    tgt = np.array([[0.25, 0.25, 0.25]])
    iso = np.array([[0.5, 0, 0, 0.5, 0, 0.5]])
    vm = oracle.VoxelMap(tgt, iso, [1.0])
    mu = np.array([[0.3, 0.3, 0.3]])
    view = np.array([0.3, 0.3, 5.0])
    up = np.array([[0.0, 0.0, 1.0]])
    away = np.array([[0.0, 0.0, -1.0]])
    side = np.array([[1.0, 0.0, 0.0]])
    for n, kept in ((up, True), (away, False), (side, True)):
        f = oracle.Factor(mu, iso, vm, nrm=n, viewpoint=view, validate=True)
        assert f.linearize(np.eye(4))["inliers"][0] == int(kept)
    # the viewpoint is expressed in the target frame and mapped back through T^-1
    T = np.eye(4)
    T[:3, 3] = [0.0, 0.0, 0.0]
    T[:3, :3] = Rotation.from_rotvec([math.pi, 0, 0]).as_matrix()
    T[:3, 3] = [0.0, 0.6, 0.6]
    f = oracle.Factor(mu, iso, vm, nrm=up, viewpoint=view, validate=True)
    tr = f.linearize(T, trace=True)
    cs = T[:3, :3].T @ (view - T[:3, 3])
    assert tr["visible"][0] == (not ((mu[0] - cs) @ up[0] > 0))


def _lm_case():
    cfg = synth.config1(seed=44, n_target=6000, n_source=1500, angle_deg=2.0, trans_m=0.2)
    f = oracle.factor_from_clouds(cfg["sources"][0], cfg["targets"][0], cfg["resolutions"])
    return f, np.asarray(cfg["poses"][0], dtype=np.float64)


@pytest.mark.parametrize("lam", [1e-4, 1.0, 30.0])
def test_lm_step_is_marquardt_damped_gauss_newton(lam):
    """One LM iteration proposes T Exp(delta) with delta = solve(H + lambda diag(H), -b) on the
    oracle's H and b (numpy solve, scipy expm); it is kept iff the error drops, and lambda is
    then divided by 10, else multiplied by 10.  At lambda = 30 the Marquardt step differs from
    the lambda*I step by far more than the tolerance, so the damping form is pinned."""
    f, T = _lm_case()
    r = f.linearize(T)
    H, b = r["H"], r["b"]
    delta = np.linalg.solve(H + lam * np.diag(np.diag(H)), -b)
    delta_eye = np.linalg.solve(H + lam * np.eye(6), -b)
    Tn = retract(T, delta)
    better = f.evaluate(Tn) < r["e"]
    out = f.lm(T, iters=1, lambda0=lam)
    assert out["e"][0] == r["e"]
    assert bool(out["accepted"][0]) == better
    if better:
        np.testing.assert_allclose(out["pose"], Tn, rtol=0, atol=1e-12)
        assert out["lambda"] == lam / 10.0
    else:
        np.testing.assert_array_equal(out["pose"], T)
        assert out["lambda"] == lam * 10.0
    if lam >= 1.0:
        assert np.linalg.norm(delta - delta_eye) > 1e3 * 1e-12 * np.linalg.norm(delta)
        assert not np.allclose(retract(T, delta_eye), Tn, rtol=0, atol=1e-9)
    assert better or lam > 1.0


def test_lm_schedule_over_iterations():
    """Ten iterations: the accept flags follow 'error drops', lambda follows /10 and x10, and
    each recorded error is the error at the pose the iteration linearized at (the expected
    poses are advanced with scipy's expm, so they agree with the oracle's to rounding)."""
    f, T = _lm_case()
    lam = 1e-4
    out = f.lm(T, iters=10, lambda0=lam)
    for it in range(10):
        r = f.linearize(T)
        assert abs(out["e"][it] - r["e"]) <= 1e-10 * r["e"], it   # poses differ by exp rounding
        delta = np.linalg.solve(r["H"] + lam * np.diag(np.diag(r["H"])), -r["b"])
        Tn = retract(T, delta)
        acc = f.evaluate(Tn) < r["e"]
        assert bool(out["accepted"][it]) == acc, it
        if acc:
            T = Tn
            lam /= 10.0
        else:
            lam *= 10.0
    assert out["lambda"] == lam
    np.testing.assert_allclose(out["pose"], T, rtol=0, atol=1e-10)


def test_lm_forced_rejects_multiply_lambda_by_ten():
    """No correspondence (H = 0: the damped system is singular) and a zero-residual optimum
    (delta = 0: the error cannot drop) both reject, keep the pose and multiply lambda by 10."""
    f, T = _lm_case()
    far = T.copy()
    far[:3, 3] += [1e4, 0.0, 0.0]
    out = f.lm(far, iters=3, lambda0=1e-4)
    assert not out["accepted"].any() and out["e"].tolist() == [0.0] * 3
    np.testing.assert_array_equal(out["pose"], far)
    assert out["lambda"] == 1e-4 * 10 * 10 * 10
    cloud, res = synth.tiny_lattice_pair(2, resolutions=(1.0,))
    vm = oracle.VoxelMap(cloud.xyz64(), cloud.cov64(), res)
    g = oracle.Factor(cloud.xyz64(), cloud.cov64(), vm)
    out = g.lm(np.eye(4), iters=2, lambda0=1e-4)
    assert out["e"].tolist() == [0.0, 0.0] and not out["accepted"].any()
    np.testing.assert_array_equal(out["pose"], np.eye(4))
    assert out["lambda"] == 1e-4 * 10 * 10
