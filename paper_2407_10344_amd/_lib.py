"""ctypes loader for ``libvgicp.so`` (argument marshalling only).

``torch`` is imported first on purpose: it loads its HIP runtime, and the
library (which needs ``libamdhip64.so.7``) then binds to that same runtime, so
torch tensors' device pointers and torch streams are valid in library calls.
"""

from __future__ import annotations

import ctypes as C
import os
import threading

import torch  # noqa: F401  (must precede loading the HIP library)

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; VGICP_LIBRARY names another build of the same sources
LIB_PATH = os.environ.get("VGICP_LIBRARY") or os.path.join(_HERE, "libvgicp.so")

VG_OK = 0
STATUS = {
    0: "VG_OK",
    -1: "VG_ERR_INVALID_ARG",
    -2: "VG_ERR_HIP",
    -3: "VG_ERR_OOM",
    -4: "VG_ERR_KEY_RANGE",
    -5: "VG_ERR_CAPACITY",
    -6: "VG_ERR_NOT_SPD",
    -7: "VG_ERR_STATE",
}

FP32_COMPENSATED = 0
FP32 = 1
FP64 = 2
PRECISIONS = {"fp32c": FP32_COMPENSATED, "fp32": FP32, "fp64": FP64}


class VGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class BatchOptions(C.Structure):
    _fields_ = [
        ("precision", C.c_int32),
        ("surface_validation", C.c_int32),
        ("use_graph", C.c_int32),
        ("plain_per_factor", C.c_int32),
        ("block_threads", C.c_int32),
        ("tile_points", C.c_int32),
        ("blocks_per_cu", C.c_int32),
        ("lane_kahan", C.c_int32),
        ("tune_cache", C.c_char_p),
        ("tile_order", C.c_int32),
    ]


# name -> (restype, argtypes); every exported symbol of include/vgicp.h
P = C.c_void_p
I32, I64, D = C.c_int32, C.c_int64, C.c_double
SIGNATURES = {
    "vg_context_create": (C.c_int, [I32, P, P]),
    "vg_context_destroy": (C.c_int, [P]),
    "vg_last_error": (C.c_char_p, []),
    "vg_version": (I32, []),
    "vg_build_voxelmap": (C.c_int, [P, P, P, I64, P, I32, P]),
    "vg_voxelmap_info": (C.c_int, [P, I32, P, P]),
    "vg_voxelmap_export": (C.c_int, [P, I32, P, P, P, P, P]),
    "vg_voxelmap_destroy": (C.c_int, [P]),
    "vg_create_source": (C.c_int, [P, P, P, P, I64, P]),
    "vg_source_set_points_async": (C.c_int, [P, P, I32]),
    "vg_source_destroy": (C.c_int, [P]),
    "vg_preprocess": (C.c_int, [P, P, I64, D, I32, P, P]),
    "vg_cloud_info": (C.c_int, [P, P, P]),
    "vg_cloud_export": (C.c_int, [P, P, P, P, P, P, P, P]),
    "vg_create_source_from_cloud": (C.c_int, [P, P, P]),
    "vg_build_voxelmap_from_cloud": (C.c_int, [P, P, P, I32, P]),
    "vg_cloud_destroy": (C.c_int, [P]),
    "vg_create_factor_batch": (C.c_int, [P, I64, P, P, P, P, P]),
    "vg_batch_info": (C.c_int, [P, P, P, P, P, P, P]),
    "vg_batch_destroy": (C.c_int, [P]),
    "vg_linearize": (C.c_int, [P, P, P, P, P, P]),
    "vg_evaluate": (C.c_int, [P, P, P]),
    "vg_overlap": (C.c_int, [P, P, P]),
    "vg_linearize_async": (C.c_int, [P, P, P, P]),
    "vg_linearize_noalloc": (C.c_int, [P, P, P, P]),
    "vg_evaluate_async": (C.c_int, [P, P, P]),
    "vg_backward_async": (C.c_int, [P, P, P, P, P, P, I32]),
    "vg_se3_retract_async": (C.c_int, [P, I64, P, P, P, P]),
    "vg_lm_run": (C.c_int, [P, P, I32, D, P, P, P]),
    "vg_lm_step_async": (C.c_int, [P, P, P, P, P]),
    "vg_batch_work": (C.c_int, [P, P, P, P]),
    "vg_correspondences": (C.c_int, [P, P, I64, P, P]),
    "vg_batch_tune": (C.c_int, [P, P, I32, P]),
    "vg_create_graph": (C.c_int, [P, I64, I64, P, P, P]),
    "vg_graph_structure": (C.c_int, [P, P, P, P]),
    "vg_graph_assemble_async": (C.c_int, [P, P, P, P, P]),
    "vg_graph_destroy": (C.c_int, [P]),
    "vg_batch_time_kernels": (C.c_int, [P, P, I32, P]),
}

_lock = threading.Lock()
_lib = None


def load(path: str = LIB_PATH):
    """Load the built library; raises if it is missing (there is no fallback)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise RuntimeError("libvgicp.so is not built (%s); run `python -m paper_2407_10344_amd.build`"
                                   % path)
            lib = C.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def last_error() -> str:
    return load().vg_last_error().decode(errors="replace")


def check(status: int):
    if status != VG_OK:
        raise VGError(status, last_error())
