"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol ``include/vgicp.h`` declares, and rejects bad handles and
arguments before touching a device."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vgicp.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(vg_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_10344_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2407_10344_amd import build
        build.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("vg_build_voxelmap", "vg_create_factor_batch", "vg_linearize", "vg_evaluate", "vg_backward_async",
              "vg_lm_run", "vg_correspondences", "vg_context_create"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2407_10344_amd import _lib
    names = declared_functions()
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares exactly the header's functions
    assert sorted(_lib.SIGNATURES) == names


def test_version_and_error_string(lib):
    assert lib.vg_version() >= 10000
    assert isinstance(lib.vg_last_error(), bytes)


def test_null_and_foreign_handles_are_rejected(lib):
    from paper_2407_10344_amd import _lib
    bogus = C.c_void_p(0)
    assert lib.vg_context_destroy(bogus) == -7
    assert lib.vg_voxelmap_destroy(bogus) == -7
    assert lib.vg_source_destroy(bogus) == -7
    assert lib.vg_batch_destroy(bogus) == -7
    assert b"invalid" in lib.vg_last_error()
    out = C.c_void_p()
    assert lib.vg_build_voxelmap(bogus, None, None, 0, None, 1, C.byref(out)) == -7
    assert lib.vg_create_factor_batch(bogus, 1, None, None, None, None, C.byref(out)) == -7
    e = (C.c_double * 1)()
    assert lib.vg_linearize(bogus, None, e, e, e, None) == -7


def test_context_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    out = C.c_void_p()
    assert lib.vg_context_create(0, None, C.byref(out)) == -2
    assert out.value is None
    assert len(lib.vg_last_error()) > 0
    assert lib.vg_context_create(0, None, None) == -1


def test_library_marks_its_calls_for_profilers():
    """The library's calls open named roctx ranges (shown by rocprofv3
    --marker-trace): it imports the range calls from the roctx library."""
    import shutil
    import subprocess
    from paper_2407_10344_amd import _lib
    nm = shutil.which("nm")
    if nm is None or not os.path.exists(_lib.LIB_PATH):
        pytest.skip("nm or the built library missing")
    out = subprocess.run([nm, "-D", _lib.LIB_PATH], capture_output=True, text=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
