"""MI355X-native batched VGICP factor linearization (GLIM, Sec. III-C).

The computation lives in ``libvgicp.so`` (HIP, gfx950) behind the C ABI of
``include/vgicp.h``; this package is its Python binding.  Importing the package
does not load the library; the first object created does, and fails loudly if
it has not been built (``python -m paper_2407_10344_amd.build``).
"""

__version__ = "1.0.0"


def __getattr__(name):
    if name in ("Context", "VoxelMap", "Source", "Cloud", "FactorBatch", "Graph", "build_workload", "poses12",
                "pose4x4"):
        from . import vgicp
        return getattr(vgicp, name)
    if name in ("VGICPCost",):
        from . import autograd
        return getattr(autograd, name)
    if name in ("VGError",):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
