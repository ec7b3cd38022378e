"""Point-cloud container, k-NN covariance preprocessing and input quantization.

Sec. III-C (Preprocessing): each point is modelled as a Gaussian whose
covariance comes from its k nearest neighbours.  As in GICP-style pipelines the
covariance is regularized by replacing its eigenvalues with (1e-3, 1, 1), so
only the smallest-eigenvalue eigenvector (the surface normal) survives.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

REG_EIGS = (1e-3, 1.0, 1.0)


@dataclass
class Cloud:
    """A Gaussian point cloud in its own frame.

    Positions are stored as ``origin + off32`` so FP64 consumers see values
    that are exactly representable as an FP64 origin plus an FP32 offset.
    """

    origin: np.ndarray          # (3,) float64, a multiple of the coarsest voxel size
    off32: np.ndarray           # (n, 3) float32 offsets from origin
    cov32: np.ndarray           # (n, 6) float32: xx, xy, xz, yy, yz, zz
    nrm32: np.ndarray           # (n, 3) float32 unit normals
    viewpoint: np.ndarray = field(default_factory=lambda: np.zeros(3))  # sensor origin, own frame

    @property
    def n(self) -> int:
        return int(self.off32.shape[0])

    def xyz64(self) -> np.ndarray:
        return self.origin[None, :] + self.off32.astype(np.float64)

    def cov64(self) -> np.ndarray:
        return self.cov32.astype(np.float64)

    def nrm64(self) -> np.ndarray:
        return self.nrm32.astype(np.float64)

    def subset(self, idx) -> "Cloud":
        return Cloud(self.origin.copy(), self.off32[idx], self.cov32[idx], self.nrm32[idx],
                     self.viewpoint.copy())


def smallest_eigvec(cov3: np.ndarray) -> np.ndarray:
    """Unit eigenvectors of the smallest eigenvalue of a stack of 3x3 symmetric matrices.

    Closed form: the eigenvalue from the trigonometric solution of the
    characteristic cubic, the vector as the longest cross product of two rows
    of (A - lambda I).  Falls back to numpy.linalg.eigh for the rare rows where
    that cross product is tiny (near-repeated smallest eigenvalue).
    """
    a, b, c = cov3[:, 0, 0], cov3[:, 1, 1], cov3[:, 2, 2]
    d, e, f = cov3[:, 0, 1], cov3[:, 0, 2], cov3[:, 1, 2]
    q = (a + b + c) / 3.0
    p1 = d * d + e * e + f * f
    p2 = (a - q) ** 2 + (b - q) ** 2 + (c - q) ** 2 + 2.0 * p1
    p = np.sqrt(np.maximum(p2 / 6.0, 1e-300))
    ba, bb, bc = (a - q) / p, (b - q) / p, (c - q) / p
    bd, be, bf = d / p, e / p, f / p
    detB = ba * (bb * bc - bf * bf) - bd * (bd * bc - bf * be) + be * (bd * bf - bb * be)
    r = np.clip(detB / 2.0, -1.0, 1.0)
    phi = np.arccos(r) / 3.0
    lam = q + 2.0 * p * np.cos(phi + 2.0 * np.pi / 3.0)
    r0 = np.stack([a - lam, d, e], axis=1)
    r1 = np.stack([d, b - lam, f], axis=1)
    r2 = np.stack([e, f, c - lam], axis=1)
    c01 = np.cross(r0, r1)
    c02 = np.cross(r0, r2)
    c12 = np.cross(r1, r2)
    n01 = np.einsum("ni,ni->n", c01, c01)
    n02 = np.einsum("ni,ni->n", c02, c02)
    n12 = np.einsum("ni,ni->n", c12, c12)
    best = np.where(n01 >= n02, np.where(n01 >= n12, 0, 2), np.where(n02 >= n12, 1, 2))
    v = np.where((best == 0)[:, None], c01, np.where((best == 1)[:, None], c02, c12))
    nv = np.sqrt(np.maximum(np.maximum(n01, n02), n12))
    scale = np.maximum(p, 1e-300) ** 2
    bad = nv < 1e-6 * scale
    out = v / np.where(nv > 0, nv, 1.0)[:, None]
    if bad.any():
        _, w = np.linalg.eigh(cov3[bad])
        out[bad] = w[:, :, 0]
    return out


def knn_cov_normals(xyz: np.ndarray, viewpoint: np.ndarray, k: int = 10, workers: int = -1):
    """k-NN covariance (self included), regularized to eigenvalues REG_EIGS.

    Returns (cov6 float64 (n,6), normals float64 (n,3)).  Normals are oriented
    toward ``viewpoint`` (n . (viewpoint - x) >= 0).
    """
    n = xyz.shape[0]
    tree = cKDTree(xyz)
    kk = min(k, n)
    _, nb = tree.query(xyz, k=kk, workers=workers)
    if kk == 1:
        nb = nb[:, None]
    nrm = np.empty((n, 3))
    step = 1 << 19
    for s in range(0, n, step):
        P = xyz[nb[s:s + step]]                  # (m, k, 3)
        mu = P.mean(axis=1)
        X = P - mu[:, None, :]
        C = np.einsum("mki,mkj->mij", X, X) / kk
        nrm[s:s + step] = smallest_eigvec(C)
    flip = np.einsum("ni,ni->n", nrm, viewpoint[None, :] - xyz) < 0
    nrm[flip] *= -1.0
    lo, hi = REG_EIGS[0], REG_EIGS[1]
    # V diag(lo, hi, hi) V^T = hi*I - (hi - lo) * n n^T
    cov = np.empty((n, 6))
    a = hi - lo
    cov[:, 0] = hi - a * nrm[:, 0] * nrm[:, 0]
    cov[:, 1] = -a * nrm[:, 0] * nrm[:, 1]
    cov[:, 2] = -a * nrm[:, 0] * nrm[:, 2]
    cov[:, 3] = hi - a * nrm[:, 1] * nrm[:, 1]
    cov[:, 4] = -a * nrm[:, 1] * nrm[:, 2]
    cov[:, 5] = hi - a * nrm[:, 2] * nrm[:, 2]
    return cov, nrm


def quantize_cloud(xyz: np.ndarray, cov: np.ndarray, nrm: np.ndarray, snap: float,
                   viewpoint=None) -> Cloud:
    """Snap the origin to a multiple of ``snap`` near the centroid and store FP32 offsets."""
    c = xyz.mean(axis=0) if xyz.shape[0] else np.zeros(3)
    origin = snap * np.round(c / snap)
    off = (xyz - origin[None, :]).astype(np.float32)
    vp = np.zeros(3) if viewpoint is None else np.asarray(viewpoint, dtype=np.float64)
    return Cloud(origin.astype(np.float64), off, cov.astype(np.float32),
                 nrm.astype(np.float32), vp)


def make_cloud(xyz: np.ndarray, viewpoint: np.ndarray, snap: float, k: int = 10,
               workers: int = -1) -> Cloud:
    cov, nrm = knn_cov_normals(xyz, viewpoint, k=k, workers=workers)
    return quantize_cloud(xyz, cov, nrm, snap, viewpoint)
