"""Python binding of the VGICP C ABI (``include/vgicp.h``): argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
numpy arrays / torch tensors to pointers, orders the library's stream against
torch's current stream for the ``*_async`` calls, and raises ``VGError`` on a
non-zero status.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import BatchOptions, PRECISIONS, check, load


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _tp(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def poses12(poses) -> np.ndarray:
    """(F, 4, 4) or (F, 12) or (4, 4) -> contiguous (F, 12) float64 [R row-major | t]."""
    P = np.asarray(poses, dtype=np.float64)
    if P.ndim == 2 and P.shape == (4, 4):
        P = P[None]
    if P.ndim == 3 and P.shape[1:] == (4, 4):
        out = np.concatenate([P[:, :3, :3].reshape(-1, 9), P[:, :3, 3]], axis=1)
    else:
        out = P.reshape(-1, 12)
    return np.ascontiguousarray(out)


def pose4x4(p12) -> np.ndarray:
    p = np.asarray(p12, dtype=np.float64).reshape(-1, 12)
    T = np.tile(np.eye(4), (p.shape[0], 1, 1))
    T[:, :3, :3] = p[:, :9].reshape(-1, 3, 3)
    T[:, :3, 3] = p[:, 9:]
    return T


class Context:
    """A device plus the HIP stream all library work is queued on."""

    def __init__(self, device: int = 0):
        lib = load()
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        h = C.c_void_p()
        check(lib.vg_context_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            torch.cuda.synchronize(self.device)
            check(load().vg_context_destroy(self.handle))
            self.handle = None

    # ordering against torch's current stream for device-pointer calls
    def enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def se3_retract(self, T0: torch.Tensor, xi: torch.Tensor, jacobian: bool = True):
        """T = T0 Exp(xi) (F x 12 FP64) and the right Jacobian J_r(xi) (F x 6 x 6) on the device."""
        F = T0.shape[0]
        T0 = T0.contiguous().to(torch.float64)
        xi = xi.contiguous().to(torch.float64)
        T = torch.empty((F, 12), dtype=torch.float64, device=T0.device)
        jr = torch.empty((F, 6, 6), dtype=torch.float64, device=T0.device) if jacobian else None
        self.enter()
        check(load().vg_se3_retract_async(self.handle, F, _tp(T0), _tp(xi), _tp(T), _tp(jr)))
        self.leave()
        return T, jr


class VoxelMap:
    """Multi-resolution Gaussian voxel map of a target cloud on the device."""

    def __init__(self, ctx: Context, xyz, cov, resolutions):
        xyz = _f64(xyz, (-1, 3))
        cov = _f64(cov, (-1, 6))
        res = _f64(resolutions, (-1,))
        self.ctx = ctx
        self.L = int(res.shape[0])
        self.resolutions = res.tolist()
        h = C.c_void_p()
        check(load().vg_build_voxelmap(ctx.handle, _p(xyz), _p(cov), xyz.shape[0], _p(res), self.L, C.byref(h)))
        self.handle = h

    @classmethod
    def from_cloud(cls, ctx: Context, cloud: "Cloud", resolutions):
        """Voxel map of a preprocessed cloud, built without leaving the device."""
        res = _f64(resolutions, (-1,))
        self = cls.__new__(cls)
        self.ctx = ctx
        self.L = int(res.shape[0])
        self.resolutions = res.tolist()
        h = C.c_void_p()
        check(load().vg_build_voxelmap_from_cloud(ctx.handle, cloud.handle, _p(res), self.L, C.byref(h)))
        self.handle = h
        return self

    def info(self, level=0):
        V, cap = C.c_int64(), C.c_int64()
        check(load().vg_voxelmap_info(self.handle, level, C.byref(V), C.byref(cap)))
        return V.value, cap.value

    def export(self, level=0):
        V, _ = self.info(level)
        keys = np.zeros((max(V, 1), 3), dtype=np.int64)
        means = np.zeros((max(V, 1), 3))
        covs = np.zeros((max(V, 1), 6))
        counts = np.zeros(max(V, 1), dtype=np.int64)
        n = C.c_int64(max(V, 1))
        check(load().vg_voxelmap_export(self.handle, level, C.byref(n), _p(keys), _p(means), _p(covs),
                                        _p(counts)))
        V = n.value
        return keys[:V], means[:V], covs[:V], counts[:V]

    def close(self):
        if self.handle:
            check(load().vg_voxelmap_destroy(self.handle))
            self.handle = None


class Source:
    """A source Gaussian cloud on the device (internally Morton ordered)."""

    def __init__(self, ctx: Context, xyz, cov, normals=None):
        xyz = _f64(xyz, (-1, 3))
        cov = _f64(cov, (-1, 6))
        nrm = None if normals is None else _f64(normals, (-1, 3))
        self.ctx = ctx
        self.n = int(xyz.shape[0])
        h = C.c_void_p()
        check(load().vg_create_source(ctx.handle, _p(xyz), _p(cov), _p(nrm), self.n, C.byref(h)))
        self.handle = h

    @classmethod
    def from_cloud(cls, ctx: Context, cloud: "Cloud"):
        """Source made from a preprocessed cloud (with its normals), on the device."""
        self = cls.__new__(cls)
        self.ctx = ctx
        self.n = cloud.n
        h = C.c_void_p()
        check(load().vg_create_source_from_cloud(ctx.handle, cloud.handle, C.byref(h)))
        self.handle = h
        return self

    def set_points(self, xyz: torch.Tensor):
        """Replace positions from a device tensor (n x 3, float32 or float64, caller order)."""
        assert xyz.is_cuda and xyz.shape == (self.n, 3)
        t = xyz.contiguous()
        dt = 0 if t.dtype == torch.float32 else 1
        if t.dtype not in (torch.float32, torch.float64):
            raise TypeError("points must be float32 or float64")
        self.ctx.enter()
        check(load().vg_source_set_points_async(self.handle, _tp(t), dt))
        self.ctx.leave()
        return t

    def close(self):
        if self.handle:
            check(load().vg_source_destroy(self.handle))
            self.handle = None


class Cloud:
    """A preprocessed frame on the device: voxel-grid downsampling, exact k-NN,
    regularised neighbour covariances and normals oriented towards the sensor."""

    def __init__(self, ctx: Context, xyz, r, k=10, sensor=(0.0, 0.0, 0.0)):
        xyz = _f64(xyz, (-1, 3))
        s = _f64(sensor, (3,))
        self.ctx = ctx
        h = C.c_void_p()
        check(load().vg_preprocess(ctx.handle, _p(xyz), xyz.shape[0], float(r), int(k), _p(s), C.byref(h)))
        self.handle = h
        m, kk = C.c_int64(), C.c_int32()
        check(load().vg_cloud_info(self.handle, C.byref(m), C.byref(kk)))
        self.n, self.k = m.value, kk.value

    def export(self):
        m, k = max(self.n, 1), self.k
        out = {"xyz": np.zeros((m, 3)), "cov": np.zeros((m, 6)), "cov_raw": np.zeros((m, 6)),
               "normals": np.zeros((m, 3)), "counts": np.zeros(m, dtype=np.int64),
               "nbr": np.zeros((m, k), dtype=np.int32), "d2": np.zeros((m, k))}
        check(load().vg_cloud_export(self.handle, _p(out["xyz"]), _p(out["cov"]), _p(out["cov_raw"]),
                                     _p(out["normals"]), _p(out["counts"]), _p(out["nbr"]), _p(out["d2"])))
        return {key: v[:self.n] for key, v in out.items()}

    def close(self):
        if self.handle:
            check(load().vg_cloud_destroy(self.handle))
            self.handle = None


class FactorBatch:
    """F factors linearized together (one upload, one download per call)."""

    def __init__(self, ctx: Context, sources, maps, viewpoints=None, precision="fp32c", validation=False,
                 use_graph=True, plain=False, block=0, tile=0, blocks_per_cu=0, lane_kahan=False,
                 tune_cache=None, tile_order=0):
        lib = load()
        self.ctx = ctx
        self.sources = list(sources)
        self.maps = list(maps)
        F = len(self.sources)
        assert F == len(self.maps) and F > 0
        self.F = F
        self.L = self.maps[0].L
        self.precision = precision
        o = BatchOptions()
        o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        o.surface_validation = int(bool(validation))
        o.use_graph = int(bool(use_graph))
        o.plain_per_factor = int(bool(plain))
        o.block_threads = int(block)
        o.tile_points = int(tile)
        o.blocks_per_cu = int(blocks_per_cu)
        o.lane_kahan = int(bool(lane_kahan))
        o.tune_cache = tune_cache.encode() if tune_cache else None
        o.tile_order = int(tile_order)
        srcs = (C.c_void_p * F)(*[s.handle.value for s in self.sources])
        tgts = (C.c_void_p * F)(*[m.handle.value for m in self.maps])
        vp = None if viewpoints is None else _f64(viewpoints, (F, 3))
        h = C.c_void_p()
        check(lib.vg_create_factor_batch(ctx.handle, F, srcs, tgts, _p(vp), C.byref(o), C.byref(h)))
        self.handle = h
        # rows of the concatenated point gradient (sources in order of first use)
        seen, self.grad_rows, self.source_rows = {}, 0, {}
        for s in self.sources:
            if id(s) not in seen:
                seen[id(s)] = self.grad_rows
                self.source_rows[id(s)] = (self.grad_rows, s.n)
                self.grad_rows += s.n

    def info(self):
        tp, nt = C.c_int64(), C.c_int64()
        bl, ti, gr, to = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(load().vg_batch_info(self.handle, C.byref(tp), C.byref(nt), C.byref(bl), C.byref(ti), C.byref(gr),
                                   C.byref(to)))
        return {"total_points": tp.value, "n_tiles": nt.value, "block_threads": bl.value,
                "tile_points": ti.value, "grid_blocks": gr.value, "tile_order": to.value}

    def linearize(self, poses):
        P = poses12(poses)
        assert P.shape[0] == self.F
        e = np.zeros(self.F)
        H = np.zeros((self.F, 6, 6))
        b = np.zeros((self.F, 6))
        inl = np.zeros((self.F, self.L), dtype=np.int64)
        check(load().vg_linearize(self.handle, _p(P), _p(e), _p(H), _p(b), _p(inl)))
        return e, H, b, inl

    def evaluate(self, poses):
        P = poses12(poses)
        e = np.zeros(self.F)
        check(load().vg_evaluate(self.handle, _p(P), _p(e)))
        return e

    def overlap(self, poses):
        """Fraction of each factor's source points that fall in an occupied target voxel (F x L)."""
        P = poses12(poses)
        o = np.zeros((self.F, self.L))
        check(load().vg_overlap(self.handle, _p(P), _p(o)))
        return o

    def linearize_async(self, d_poses: torch.Tensor, out: torch.Tensor = None, inliers: torch.Tensor = None):
        """e/H/b rows (F x 43 FP64) and inlier counts (F x L int64) on the device,
        stream-ordered; out / inliers: caller tensors to reuse (else new ones)."""
        d_poses = d_poses.contiguous()
        if out is None:
            out = torch.empty((self.F, 43), dtype=torch.float64, device=d_poses.device)
        if inliers is None:
            inliers = torch.empty((self.F, self.L), dtype=torch.int64, device=d_poses.device)
        assert out.is_contiguous() and out.dtype == torch.float64 and out.shape == (self.F, 43)
        assert inliers.is_contiguous() and inliers.dtype == torch.int64 and inliers.shape == (self.F, self.L)
        inl = inliers
        self.ctx.enter()
        check(load().vg_linearize_async(self.handle, _tp(d_poses), _tp(out), _tp(inl)))
        self.ctx.leave()
        return out, inl

    def linearize_noalloc(self, d_poses: torch.Tensor, out: torch.Tensor, inliers: torch.Tensor = None):
        """vg_linearize_async's results into caller-provided device tensors (F x 43 FP64,
        F x L int64 or None), with the kernels' scratch in the library's fixed array."""
        d_poses = d_poses.contiguous()
        assert out.is_contiguous() and out.dtype == torch.float64 and out.shape == (self.F, 43)
        assert inliers is None or (inliers.is_contiguous() and inliers.dtype == torch.int64
                                   and inliers.shape == (self.F, self.L))
        self.ctx.enter()
        check(load().vg_linearize_noalloc(self.handle, _tp(d_poses), _tp(out), _tp(inliers)))
        self.ctx.leave()
        return out, inliers

    def evaluate_async(self, d_poses: torch.Tensor):
        d_poses = d_poses.contiguous()
        e = torch.empty(self.F, dtype=torch.float64, device=d_poses.device)
        self.ctx.enter()
        check(load().vg_evaluate_async(self.handle, _tp(d_poses), _tp(e)))
        self.ctx.leave()
        return e

    def backward_async(self, d_poses: torch.Tensor, grad_e: torch.Tensor, jr=None, points_dtype=None):
        """(grad_xi F x 6 FP64, grad_points grad_rows x 3 or None)."""
        d_poses = d_poses.contiguous()
        grad_e = grad_e.contiguous().to(torch.float64)
        gxi = torch.empty((self.F, 6), dtype=torch.float64, device=d_poses.device)
        gp = None
        dt = 0
        if points_dtype is not None:
            gp = torch.empty((self.grad_rows, 3), dtype=points_dtype, device=d_poses.device)
            dt = 0 if points_dtype == torch.float32 else 1
        jr_c = None if jr is None else jr.contiguous()
        self.ctx.enter()
        check(load().vg_backward_async(self.handle, _tp(d_poses), _tp(grad_e), _tp(jr_c), _tp(gxi), _tp(gp), dt))
        self.ctx.leave()
        return gxi, gp

    def lm(self, poses, iters=10, lambda0=1e-4):
        P = poses12(poses)
        out = np.zeros_like(P)
        acc = np.zeros((self.F, iters), dtype=np.int32)
        eh = np.zeros((self.F, iters))
        check(load().vg_lm_run(self.handle, _p(P), iters, float(lambda0), _p(out), _p(acc), _p(eh)))
        return pose4x4(out), acc.astype(bool), eh

    def lm_step_async(self, d_poses: torch.Tensor, d_lambda: torch.Tensor, want_e=True, want_accepted=True):
        """One device LM iteration in place on (F x 12) poses and (F) lambda (FP64 tensors);
        returns (e at the input poses, accepted flags) as device tensors (or None)."""
        assert d_poses.dtype == torch.float64 and d_poses.is_contiguous() and d_poses.shape == (self.F, 12)
        assert d_lambda.dtype == torch.float64 and d_lambda.is_contiguous() and d_lambda.shape == (self.F,)
        e = torch.empty(self.F, dtype=torch.float64, device=d_poses.device) if want_e else None
        acc = torch.empty(self.F, dtype=torch.int32, device=d_poses.device) if want_accepted else None
        self.ctx.enter()
        check(load().vg_lm_step_async(self.handle, _tp(d_poses), _tp(d_lambda), _tp(e), _tp(acc)))
        self.ctx.leave()
        return e, acc

    def work(self):
        """Work of the last linearize / evaluate / overlap: (walked points F, walked chunks F,
        table lookups F x L)."""
        wp = np.zeros(self.F, dtype=np.int64)
        wc = np.zeros(self.F, dtype=np.int64)
        lk = np.zeros((self.F, self.L), dtype=np.int64)
        check(load().vg_batch_work(self.handle, _p(wp), _p(wc), _p(lk)))
        return wp, wc, lk

    def correspondences(self, pose, factor):
        P = poses12(pose)[0]
        n = self.sources[factor].n
        keys = np.zeros((max(n, 1), self.L, 3), dtype=np.int64)
        found = np.zeros((max(n, 1), self.L), dtype=np.int32)
        check(load().vg_correspondences(self.handle, _p(P), int(factor), _p(keys), _p(found)))
        return keys[:n], found[:n]

    def tune(self, poses, reps=3):
        P = poses12(poses)
        ch = np.zeros(4, dtype=np.int32)
        check(load().vg_batch_tune(self.handle, _p(P), int(reps), _p(ch)))
        return {"block_threads": int(ch[0]), "tile_points": int(ch[1]), "blocks_per_cu": int(ch[2]),
                "tile_order": int(ch[3])}

    def time_kernels(self, poses, reps=10):
        P = poses12(poses)
        ms = np.zeros(3, dtype=np.float32)
        check(load().vg_batch_time_kernels(self.handle, _p(P), int(reps), _p(ms)))
        return {"tile_kernel_ms": float(ms[0]), "reduce_ms": float(ms[1]), "call_ms": float(ms[2])}

    def close(self):
        if self.handle:
            check(load().vg_batch_destroy(self.handle))
            self.handle = None


class Graph:
    """Pose graph over N nodes: expands linearized factors into two-node blocks and
    assembles the block-sparse (BSR, 6x6 blocks) normal equations on the device."""

    def __init__(self, ctx: Context, N, node_i, node_j):
        ni = np.ascontiguousarray(node_i, dtype=np.int64)
        nj = np.ascontiguousarray(node_j, dtype=np.int64)
        self.ctx = ctx
        self.N, self.F = int(N), int(ni.shape[0])
        h = C.c_void_p()
        check(load().vg_create_graph(ctx.handle, self.N, self.F, _p(ni), _p(nj), C.byref(h)))
        self.handle = h
        nnzb = C.c_int64()
        check(load().vg_graph_structure(self.handle, C.byref(nnzb), None, None))
        self.nnzb = nnzb.value
        self.row_ptr = np.zeros(self.N + 1, dtype=np.int64)
        self.col_idx = np.zeros(max(self.nnzb, 1), dtype=np.int64)
        check(load().vg_graph_structure(self.handle, None, _p(self.row_ptr), _p(self.col_idx)))
        self.col_idx = self.col_idx[:self.nnzb]

    def assemble(self, d_poses: torch.Tensor, d_lin: torch.Tensor):
        """(values nnzb x 6 x 6, rhs N x 6) FP64 device tensors."""
        values = torch.empty((self.nnzb, 6, 6), dtype=torch.float64, device=d_lin.device)
        rhs = torch.empty((self.N, 6), dtype=torch.float64, device=d_lin.device)
        d_poses = d_poses.contiguous()
        d_lin = d_lin.contiguous()
        self.ctx.enter()
        check(load().vg_graph_assemble_async(self.handle, _tp(d_poses), _tp(d_lin), _tp(values), _tp(rhs)))
        self.ctx.leave()
        return values, rhs

    def dense(self, values, rhs):
        """Dense (6N x 6N, 6N) host copies, for checks on small graphs."""
        v = values.cpu().numpy()
        Hd = np.zeros((6 * self.N, 6 * self.N))
        for r in range(self.N):
            for k in range(self.row_ptr[r], self.row_ptr[r + 1]):
                c = self.col_idx[k]
                Hd[6 * r:6 * r + 6, 6 * c:6 * c + 6] = v[k]
        return Hd, rhs.cpu().numpy().reshape(-1)

    def close(self):
        if self.handle:
            check(load().vg_graph_destroy(self.handle))
            self.handle = None


def build_workload(ctx: Context, cfg: dict, precision="fp32c", validation=False, use_graph=True, plain=False,
                   **shape):
    """Device objects for a ``synth`` workload dict: (maps, sources, batch)."""
    res = cfg["resolutions"]
    tgt_ids = sorted({t for (_, t) in cfg["factors"]})
    src_ids = sorted({s for (s, _) in cfg["factors"]})
    maps = {t: VoxelMap(ctx, cfg["targets"][t].xyz64(), cfg["targets"][t].cov64(), res) for t in tgt_ids}
    srcs = {s: Source(ctx, cfg["sources"][s].xyz64(), cfg["sources"][s].cov64(), cfg["sources"][s].nrm64())
            for s in src_ids}
    batch = FactorBatch(ctx, [srcs[s] for (s, _) in cfg["factors"]], [maps[t] for (_, t) in cfg["factors"]],
                        viewpoints=np.asarray(cfg["target_viewpoints"]), precision=precision,
                        validation=validation, use_graph=use_graph, plain=plain, **shape)
    return maps, srcs, batch
