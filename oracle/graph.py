"""Two-node expansion and dense normal-equation assembly -- TEST INFRASTRUCTURE.

GLIM Sec. III-C: a matching-cost factor between poses T_i (source) and T_j
(target) yields H_ii, H_ij, H_jj, b_i, b_j.  The factor is linearized w.r.t.
a right perturbation of its relative pose T = T_j^-1 T_i; perturbing the two
absolute poses on the right, T_j^-1 Exp(-xi_j) ... gives the relative tangent
xi = xi_i - Ad(T^-1) xi_j to first order, hence (A = Ad(T^-1)):
    H_ii = H, H_ij = -H A, H_jj = A^T H A, b_i = b, b_j = -A^T b.
This module writes those products out with explicit 6x6 matrices (numpy, FP64).
"""

from __future__ import annotations

import numpy as np


def hat(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def adjoint(T):
    """Ad_T for xi = [omega; v]: [[R, 0], [(t)x R, R]]."""
    T = np.asarray(T, dtype=np.float64)
    Rm, t = T[:3, :3], T[:3, 3]
    A = np.zeros((6, 6))
    A[:3, :3] = Rm
    A[3:, 3:] = Rm
    A[3:, :3] = hat(t) @ Rm
    return A


def expand(H, b, T):
    """(H_ii, H_ij, H_jj, b_i, b_j) of one factor with relative pose T = T_j^-1 T_i."""
    A = adjoint(np.linalg.inv(T))
    Hij = -H @ A
    return H.copy(), Hij, A.T @ H @ A, b.copy(), -A.T @ b


def assemble_dense(N, node_i, node_j, Hs, bs, Ts):
    """Dense 6N x 6N normal matrix and 6N right-hand side of a pose graph."""
    Hd = np.zeros((6 * N, 6 * N))
    bd = np.zeros(6 * N)
    for f, (i, j) in enumerate(zip(node_i, node_j)):
        Hii, Hij, Hjj, bi, bj = expand(Hs[f], bs[f], Ts[f])
        si, sj = slice(6 * i, 6 * i + 6), slice(6 * j, 6 * j + 6)
        Hd[si, si] += Hii
        Hd[si, sj] += Hij
        Hd[sj, si] += Hij.T
        Hd[sj, sj] += Hjj
        bd[si] += bi
        bd[sj] += bj
    return Hd, bd
