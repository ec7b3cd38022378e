"""FP64 CPU oracle for VGICP factor linearization -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The device library never does, and
nothing here imports the device library: the two share no code.

The arithmetic lives in ``vgicp_oracle.c`` (plain C, FP64, no threading); this
module only compiles it with gcc and marshals numpy arrays through ctypes.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vgicp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Level(C.Structure):
    _fields_ = [("r", C.c_double), ("n", C.c_int64), ("key", C.c_void_p), ("mean", C.c_void_p),
                ("cov", C.c_void_p)]


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("xyz", C.c_void_p), ("cov", C.c_void_p), ("nrm", C.c_void_p),
                ("L", C.c_int32), ("levels", C.c_void_p), ("viewpoint", C.c_void_p),
                ("validate", C.c_int32), ("frozen", C.c_void_p), ("omega_pose", C.c_void_p)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(build())
            P = C.c_void_p
            L.orc_voxelize.restype = C.c_int64
            L.orc_voxelize.argtypes = [P, P, C.c_int64, C.c_double, P, P, P, P]
            L.orc_lookup.restype = C.c_int64
            L.orc_lookup.argtypes = [P, P]
            L.orc_linearize.restype = C.c_int
            L.orc_linearize.argtypes = [P, P, P, P, P, P, P, P, P, P]
            L.orc_point_terms.restype = C.c_int
            L.orc_point_terms.argtypes = [P, P, C.c_int64, C.c_int32, P, P]
            L.orc_evaluate.restype = C.c_int
            L.orc_evaluate.argtypes = [P, P, P]
            L.orc_gradient_scale.restype = C.c_int
            L.orc_gradient_scale.argtypes = [P, P, P]
            L.orc_gradient.restype = C.c_int
            L.orc_gradient.argtypes = [P, P, P, P]
            L.orc_se3_exp.restype = None
            L.orc_se3_exp.argtypes = [P, P]
            L.orc_pose_mul.restype = None
            L.orc_pose_mul.argtypes = [P, P, P]
            L.orc_lm.restype = C.c_int
            L.orc_lm.argtypes = [P, P, C.c_int32, C.c_double, P, P, P, P]
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def as_pose12(T) -> np.ndarray:
    T = np.asarray(T, dtype=np.float64)
    if T.shape == (4, 4):
        return np.concatenate([T[:3, :3].reshape(-1), T[:3, 3]])
    return np.ascontiguousarray(T.reshape(12))


def pose12_to_4x4(p) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = np.asarray(p[:9]).reshape(3, 3)
    T[:3, 3] = p[9:12]
    return T


def voxelize(xyz, cov, r):
    """One voxel-map level: (keys (V,3) int64, means (V,3), covs (V,6), counts (V,))."""
    xyz = _f64(xyz, (-1, 3))
    cov = _f64(cov, (-1, 6))
    n = xyz.shape[0]
    key = np.empty((max(n, 1), 3), dtype=np.int64)
    mean = np.empty((max(n, 1), 3))
    cv = np.empty((max(n, 1), 6))
    cnt = np.empty(max(n, 1), dtype=np.int64)
    V = lib().orc_voxelize(_p(xyz), _p(cov), n, float(r), _p(key), _p(mean), _p(cv), _p(cnt))
    if V < 0:
        raise RuntimeError("orc_voxelize failed")
    return key[:V].copy(), mean[:V].copy(), cv[:V].copy(), cnt[:V].copy()


class VoxelMap:
    """Multi-resolution Gaussian voxel map of a target cloud (one level per resolution)."""

    def __init__(self, xyz, cov, resolutions):
        self.resolutions = [float(r) for r in resolutions]
        self.levels = [voxelize(xyz, cov, r) for r in self.resolutions]
        self._structs = (_Level * len(self.levels))()
        for i, (r, (k, m, c, _)) in enumerate(zip(self.resolutions, self.levels)):
            self._structs[i] = _Level(r, k.shape[0], _p(k), _p(m), _p(c))

    @property
    def L(self):
        return len(self.levels)


class Factor:
    """One VGICP factor: a source Gaussian cloud matched into a target voxel map."""

    def __init__(self, xyz, cov, vmap: VoxelMap, nrm=None, viewpoint=None, validate=False):
        self.xyz = _f64(xyz, (-1, 3))
        self.cov = _f64(cov, (-1, 6))
        self.nrm = None if nrm is None else _f64(nrm, (-1, 3))
        self.vmap = vmap
        self.viewpoint = _f64(np.zeros(3) if viewpoint is None else viewpoint, (3,))
        self.validate = bool(validate)
        if self.validate and self.nrm is None:
            raise ValueError("validation needs normals")

    @property
    def n(self):
        return self.xyz.shape[0]

    def _problem(self, frozen=None, omega_pose=None):
        keep = []
        fz = None
        if frozen is not None:
            fz = np.ascontiguousarray(frozen, dtype=np.int64).reshape(self.n, self.vmap.L)
            keep.append(fz)
        op = None
        if omega_pose is not None:
            op = as_pose12(omega_pose)
            keep.append(op)
        pr = _Problem(self.n, _p(self.xyz), _p(self.cov), _p(self.nrm), self.vmap.L,
                      C.addressof(self.vmap._structs), _p(self.viewpoint), int(self.validate),
                      _p(fz), _p(op))
        return pr, keep

    def linearize(self, pose, trace=False, frozen=None, omega_pose=None):
        pr, keep = self._problem(frozen, omega_pose)
        T = as_pose12(pose)
        e = np.zeros(1)
        H = np.zeros(36)
        b = np.zeros(6)
        inl = np.zeros(self.vmap.L, dtype=np.int64)
        n, L = self.n, self.vmap.L
        tk = tv = tf = tvis = None
        if trace:
            tk = np.empty((n, L, 3), dtype=np.int64)
            tv = np.empty((n, L), dtype=np.int64)
            tf = np.empty((n, L))
            tvis = np.empty(n, dtype=np.int32)
        st = lib().orc_linearize(C.byref(pr), _p(T), _p(e), _p(H), _p(b), _p(inl), _p(tk), _p(tv),
                                 _p(tf), _p(tvis))
        if st != 0:
            raise RuntimeError("orc_linearize failed: %d" % st)
        out = {"e": float(e[0]), "H": H.reshape(6, 6), "b": b, "inliers": inl}
        if trace:
            out.update(keys=tk, vidx=tv, face=tf, visible=tvis.astype(bool))
        return out

    def point_terms(self, pose, k, level, key):
        pr, keep = self._problem()
        T = as_pose12(pose)
        kk = np.ascontiguousarray(key, dtype=np.int64).reshape(3)
        out = np.zeros(43)
        st = lib().orc_point_terms(C.byref(pr), _p(T), int(k), int(level), _p(kk), _p(out))
        if st < 0:
            raise RuntimeError("orc_point_terms failed: %d" % st)
        return bool(st), out[0], out[1:37].reshape(6, 6), out[37:43]

    def gradient_scale(self, pose):
        """(sum over matched pairs of |b_k| of the rotation half, the same of the
        translation half): the scale of b's summands, against which the error of a
        sum that cancels is stated."""
        pr, keep = self._problem()
        T = as_pose12(pose)
        out = np.zeros(2)
        st = lib().orc_gradient_scale(C.byref(pr), _p(T), _p(out))
        if st != 0:
            raise RuntimeError("orc_gradient_scale failed: %d" % st)
        return float(out[0]), float(out[1])

    def evaluate(self, pose, frozen=None, omega_pose=None):
        pr, keep = self._problem(frozen, omega_pose)
        T = as_pose12(pose)
        e = np.zeros(1)
        st = lib().orc_evaluate(C.byref(pr), _p(T), _p(e))
        if st != 0:
            raise RuntimeError("orc_evaluate failed: %d" % st)
        return float(e[0])

    def gradient(self, pose, frozen=None, points=True):
        pr, keep = self._problem(frozen)
        T = as_pose12(pose)
        g = np.zeros(6)
        gm = np.zeros((self.n, 3)) if points else None
        st = lib().orc_gradient(C.byref(pr), _p(T), _p(g), _p(gm))
        if st != 0:
            raise RuntimeError("orc_gradient failed: %d" % st)
        return g, gm

    def lm(self, pose, iters=10, lambda0=1e-4):
        pr, keep = self._problem()
        T = as_pose12(pose)
        out = np.zeros(12)
        acc = np.zeros(iters, dtype=np.int32)
        eh = np.zeros(iters)
        lam = np.zeros(1)
        st = lib().orc_lm(C.byref(pr), _p(T), int(iters), float(lambda0), _p(out), _p(acc), _p(eh),
                          _p(lam))
        if st != 0:
            raise RuntimeError("orc_lm failed: %d" % st)
        return {"pose": pose12_to_4x4(out), "accepted": acc.astype(bool), "e": eh,
                "lambda": float(lam[0])}


def se3_exp(xi) -> np.ndarray:
    x = _f64(xi, (6,))
    out = np.zeros(12)
    lib().orc_se3_exp(_p(x), _p(out))
    return pose12_to_4x4(out)


def factor_from_clouds(source, target, resolutions, viewpoint=None, validate=False, vmap=None):
    """Oracle factor from two ``synth.Cloud`` objects (FP64 values of the same inputs)."""
    vm = vmap or VoxelMap(target.xyz64(), target.cov64(), resolutions)
    return Factor(source.xyz64(), source.cov64(), vm, nrm=source.nrm64(), viewpoint=viewpoint,
                  validate=validate)
