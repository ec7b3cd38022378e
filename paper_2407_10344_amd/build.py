"""Build ``libvgicp.so`` (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_2407_10344_amd.build`` (always recompiles).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libvgicp.so")
BUILD = os.path.join(PKG, "_build")

SOURCES = ["vg_api.cpp", "vg_voxelmap.hip", "vg_factor.hip", "vg_lm.hip", "vg_graph.hip", "vg_preprocess.hip"]

# per-source flags: the preprocessing file forms squared distances that decide
# neighbour ranks with each operation rounded on its own, so nothing there may
# be contracted into fused multiply-adds
SOURCE_FLAGS = {"vg_preprocess.hip": ["-ffp-contract=off"]}

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "--offload-arch=gfx950",
    "-mcode-object-version=5",
    # no packed-FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-fast-math",
    "-ffp-contract=fast",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
    "-Wno-unused-but-set-variable",
    "-I" + INCLUDE,
    "-I" + CSRC,
]


def _compile(src: str, extra=()) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    flags = [f for f in FLAGS if not (f.startswith("-ffp-contract") and src in SOURCE_FLAGS)]
    flags += SOURCE_FLAGS.get(src, [])
    cmd = [HIPCC, *flags, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *flags, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-8000:]))
    return obj


def build(verbose: bool = False, extra=(), out: str = OUT) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    tmp = out + ".tmp%d" % os.getpid()
    # roctx: the named ranges around the library's calls (rocprofv3 --marker-trace)
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs,
           "-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-8000:])
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    args = sys.argv[1:]
    out = OUT
    if "--out" in args:
        i = args.index("--out")
        out = os.path.abspath(args[i + 1])
        del args[i:i + 2]
    build(verbose=True, extra=args, out=out)
