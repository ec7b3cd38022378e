"""Pins of the two-node expansion / dense assembly (oracle/graph.py).

The graph-level cost E(xi_1..xi_N) = sum_f e_f(T_j(xi_j)^-1 T_i(xi_i)) is
evaluated through the FP64 oracle with correspondences and W frozen; its
central finite differences fix the assembled right-hand side (b = 1/2 dE/dxi)
and, at zero residual, the assembled normal matrix (H = 1/2 d2E/dxi2).
"""

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import synth
from oracle.graph import adjoint, assemble_dense, expand


def twist(xi):
    w, v = xi[:3], xi[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    X[:3, 3] = v
    return X


def make_graph(noise, seed):
    """3 nodes seeing the same one-point-per-voxel lattice, factors 0->1, 1->2, 2->0, 0->2."""
    cloud, res = synth.tiny_lattice_pair(seed, resolutions=(1.0,))
    rng = np.random.default_rng(seed)
    world = cloud.xyz64()
    Tabs = [np.eye(4)] + [expm(twist(rng.normal(size=6) * 0.02)) for _ in range(2)]
    # cloud of node n expressed in its own frame (+ optional noise)
    clouds = []
    for T in Tabs:
        Ti = np.linalg.inv(T)
        pts = world @ Ti[:3, :3].T + Ti[:3, 3] + rng.normal(scale=noise, size=world.shape)
        R = Ti[:3, :3]
        C = cloud.cov64()
        M = np.stack([C[:, [0, 1, 2]], C[:, [1, 3, 4]], C[:, [2, 4, 5]]], axis=1)
        M2 = R[None] @ M @ R.T[None]
        cv = np.stack([M2[:, 0, 0], M2[:, 0, 1], M2[:, 0, 2], M2[:, 1, 1], M2[:, 1, 2], M2[:, 2, 2]], axis=1)
        clouds.append((pts, cv))
    edges = [(0, 1), (1, 2), (2, 0), (0, 2)]
    maps = [oracle.VoxelMap(p, c, res) for (p, c) in clouds]
    factors = [oracle.Factor(clouds[i][0], clouds[i][1], maps[j]) for (i, j) in edges]
    return Tabs, edges, factors


def rel(Tabs, i, j):
    return np.linalg.inv(Tabs[j]) @ Tabs[i]


@pytest.mark.parametrize("noise", [0.0, 0.03])
def test_assembled_rhs_is_half_gradient(noise):
    Tabs, edges, factors = make_graph(noise, 1)
    N = len(Tabs)
    Ts = [rel(Tabs, i, j) for (i, j) in edges]
    lin = [f.linearize(T) for f, T in zip(factors, Ts)]
    frozen = [f.linearize(T, trace=True)["vidx"] for f, T in zip(factors, Ts)]
    Hd, bd = assemble_dense(N, [i for i, _ in edges], [j for _, j in edges], [r["H"] for r in lin],
                            [r["b"] for r in lin], Ts)

    def E(xi):
        Tp = [T @ expm(twist(xi[6 * n:6 * n + 6])) for n, T in enumerate(Tabs)]
        return sum(f.evaluate(np.linalg.inv(Tp[j]) @ Tp[i], frozen=fz, omega_pose=T0)
                   for f, (i, j), fz, T0 in zip(factors, edges, frozen, Ts))

    h = 1e-6
    g = np.zeros(6 * N)
    for k in range(6 * N):
        d = np.zeros(6 * N)
        d[k] = h
        g[k] = (E(d) - E(-d)) / (2 * h)
    if noise == 0.0:
        assert np.abs(bd).max() < 1e-10
    np.testing.assert_allclose(bd, g / 2, rtol=1e-5, atol=1e-7 * max(1.0, np.abs(g).max()))


def test_assembled_matrix_is_half_hessian_at_zero_residual():
    Tabs, edges, factors = make_graph(0.0, 2)
    N = len(Tabs)
    Ts = [rel(Tabs, i, j) for (i, j) in edges]
    lin = [f.linearize(T) for f, T in zip(factors, Ts)]
    frozen = [f.linearize(T, trace=True)["vidx"] for f, T in zip(factors, Ts)]
    Hd, _ = assemble_dense(N, [i for i, _ in edges], [j for _, j in edges], [r["H"] for r in lin],
                           [r["b"] for r in lin], Ts)

    def E(xi):
        Tp = [T @ expm(twist(xi[6 * n:6 * n + 6])) for n, T in enumerate(Tabs)]
        return sum(f.evaluate(np.linalg.inv(Tp[j]) @ Tp[i], frozen=fz)
                   for f, (i, j), fz in zip(factors, edges, frozen))

    h = 1e-4
    D = 6 * N
    Hfd = np.zeros((D, D))
    I = np.eye(D) * h
    for a in range(D):
        for c in range(a, D):
            v = (E(I[a] + I[c]) - E(I[a] - I[c]) - E(-I[a] + I[c]) + E(-I[a] - I[c])) / (4 * h * h)
            Hfd[a, c] = Hfd[c, a] = v
    np.testing.assert_allclose(Hd, Hfd / 2, rtol=1e-4, atol=1e-5 * np.abs(Hd).max())
    # gauge freedom: a common motion of all nodes leaves E unchanged -> H has a 6-d null space
    w = np.linalg.eigvalsh(Hd)
    assert np.sum(np.abs(w) < 1e-8 * w.max()) == 6


def test_adjoint_identity():
    """Ad maps right tangents through a pose: T Exp(xi) = Exp(Ad_T xi) T."""
    rng = np.random.default_rng(0)
    T = expm(twist(rng.normal(size=6)))
    xi = rng.normal(size=6) * 0.1
    np.testing.assert_allclose(T @ expm(twist(xi)), expm(twist(adjoint(T) @ xi)) @ T, atol=1e-12)
    H = rng.normal(size=(6, 6))
    H = H @ H.T
    b = rng.normal(size=6)
    Hii, Hij, Hjj, bi, bj = expand(H, b, T)
    np.testing.assert_allclose(Hjj, Hjj.T, atol=1e-12)
    np.testing.assert_allclose(bi + np.linalg.inv(adjoint(np.linalg.inv(T))).T @ bj, 0, atol=1e-12)
