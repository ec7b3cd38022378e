"""Seeded synthetic inputs for batched VGICP factor linearization.

This package is shared by the FP64 oracle tests and by the device path.  It
holds none of the factor's arithmetic (no voxelization, no transform of a
source cloud by a factor pose, no residuals): it only produces point clouds,
their per-point k-NN covariances and normals (computed with scipy's k-d tree,
as input construction for the factor path), raw LiDAR frames, and the
relative poses at which factors are linearized.  The device preprocessing
(downsampling, k-NN, covariances) and its oracle use none of this package's
covariance code: they start from the raw frames.

Every array that crosses into the oracle or the device library is FP64 whose
values are exactly ``origin + float32 offset`` (positions) or exactly float32
(covariances, normals), so both sides see identical inputs.
"""

from .clouds import Cloud, quantize_cloud
from .configs import (
    config1,
    config2,
    config3,
    config3_factor_list,
    config3_submap,
    config4,
    config5,
    tiny_lattice_pair,
    random_pose,
    raw_frame,
    thin_wall_pair,
    local_mapping,
)

__all__ = [
    "Cloud",
    "quantize_cloud",
    "config1",
    "config2",
    "config3",
    "config3_factor_list",
    "config3_submap",
    "config4",
    "config5",
    "tiny_lattice_pair",
    "random_pose",
    "raw_frame",
    "thin_wall_pair",
    "local_mapping",
]
