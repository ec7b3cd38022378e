"""Point-cloud preprocessing, plain FP64 definition -- TEST INFRASTRUCTURE.

GLIM Sec. III-C (Preprocessing) and Sec. IV-A: every input point becomes a
Gaussian (mu_k, C_k) whose covariance comes from its k nearest neighbours;
the frame is downsampled first and the exact k-NN search is done once per
frame.  The paper fixes neither the downsampling method nor the covariance
normalisation nor the regularisation; the readings taken here:

* downsampling: voxel grid of size r, one output point per occupied voxel,
  the mean of its input points (sums in input order), outputs in ascending
  lexicographic order of the integer voxel key floor(x / r);
* k-NN: the k nearest downsampled points of each downsampled point, itself
  included; squared distance ((dx*dx + dy*dy) + dz*dz) with every operation
  rounded separately; ties by the smaller index; fewer than k points -> all;
* covariance: (1/k) sum (p_j - pbar)(p_j - pbar)^T over the neighbours;
* regularisation (plane-to-plane GICP): eigenvalues replaced by
  (eps, 1, 1) in ascending order, eps = 1e-3, i.e. C = I - (1 - eps) n n^T;
* normal n: eigenvector of the smallest eigenvalue, oriented so that
  n . (sensor - p) >= 0.

Plain numpy, no blocking beyond what memory needs.  knn() is brute force;
knn_tree() takes the neighbours from scipy's k-d tree (a library search
primitive, pinned against knn()) for clouds where brute force is too slow.
"""

from __future__ import annotations

import numpy as np

EPS = 1e-3


def downsample(xyz, r):
    """Voxel-grid centroids.  Returns (centroids m x 3, keys m x 3 int64, counts m)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    if len(xyz) == 0:
        return np.zeros((0, 3)), np.zeros((0, 3), np.int64), np.zeros(0, np.int64)
    keys = np.floor(xyz / r).astype(np.int64)
    uk, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(-1)
    sums = np.zeros((len(uk), 3))
    # sequential accumulation in input order (np.add.at is unbuffered, element by element)
    np.add.at(sums, inv, xyz)
    return sums / cnt[:, None], uk, cnt


def sqdist(p, q):
    """Squared distances from one point p to rows q, each operation rounded."""
    dx = q[:, 0] - p[0]
    dy = q[:, 1] - p[1]
    dz = q[:, 2] - p[2]
    return (dx * dx + dy * dy) + dz * dz


def knn(points, k, queries=None):
    """Exact k nearest neighbours by brute force (index, squared distance) per query.

    Returns (idx q x k int64, d2 q x k) sorted by (distance, index); rows of a
    cloud with fewer than k points are padded with -1 / inf.
    """
    P = np.asarray(points, dtype=np.float64)
    qs = np.arange(len(P)) if queries is None else np.asarray(queries, dtype=np.int64)
    kk = min(k, len(P))
    idx = np.full((len(qs), k), -1, np.int64)
    d2 = np.full((len(qs), k), np.inf)
    order_idx = np.arange(len(P))
    for row, i in enumerate(qs):
        d = sqdist(P[i], P)
        o = np.lexsort((order_idx, d))[:kk]
        idx[row, :kk] = o
        d2[row, :kk] = d[o]
    return idx, d2


def knn_tree(points, k):
    """The same k nearest neighbours from scipy's k-d tree (a library search
    primitive; exact).  Rows are ordered by (distance, index) like knn(); it
    differs from knn() only where distances tie at the k-th place, which
    continuous random data does not produce.  Used where brute force is too slow."""
    from scipy.spatial import cKDTree
    P = np.asarray(points, dtype=np.float64)
    kk = min(k, len(P))
    idx = np.full((len(P), k), -1, np.int64)
    d2 = np.full((len(P), k), np.inf)
    if kk == 0:
        return idx, d2
    _, nb = cKDTree(P).query(P, k=kk)
    nb = nb.reshape(len(P), kk)
    for row in range(len(P)):
        d = sqdist(P[row], P[nb[row]])
        o = np.lexsort((nb[row], d))
        idx[row, :kk] = nb[row][o]
        d2[row, :kk] = d[o]
    return idx, d2


def covariance(points, nbr):
    """(1/k) sum (p - pbar)(p - pbar)^T over the valid neighbours of each row."""
    P = np.asarray(points, dtype=np.float64)
    out = np.zeros((len(nbr), 3, 3))
    for row, ids in enumerate(nbr):
        ids = ids[ids >= 0]
        Q = P[ids]
        m = Q.mean(axis=0)
        D = Q - m
        out[row] = D.T @ D / len(ids)
    return out


def regularize(C, xyz, sensor):
    """Plane-to-plane regularisation and oriented normals.

    Returns (C_reg n x 3 x 3, normals n x 3, eigenvalues n x 3 ascending).
    """
    w, V = np.linalg.eigh(C)
    n = V[:, :, 0].copy()
    flip = np.einsum("ni,ni->n", n, np.asarray(sensor)[None] - xyz) < 0
    n[flip] *= -1
    Creg = np.einsum("nij,j,nkj->nik", V, np.array([EPS, 1.0, 1.0]), V)
    return Creg, n, w


def preprocess(xyz, r, k, sensor, search=None):
    """Downsample, k-NN, covariance, regularisation.  Returns a dict of the stages.
    search: None = brute force (knn), "tree" = knn_tree."""
    c, keys, cnt = downsample(xyz, r)
    idx, d2 = knn_tree(c, k) if search == "tree" else knn(c, k)
    C = covariance(c, idx)
    Creg, n, w = regularize(C, c, sensor)
    return {"xyz": c, "keys": keys, "counts": cnt, "nbr": idx, "d2": d2, "cov_raw": C, "cov": Creg,
            "normals": n, "eig": w}


def cov6(C):
    """3x3 -> (xx, xy, xz, yy, yz, zz)."""
    return np.stack([C[:, 0, 0], C[:, 0, 1], C[:, 0, 2], C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]], axis=1)
