"""The parity helpers (oracle/parity.py) on the oracle alone: with the oracle's own
correspondences the frozen evaluation reproduces the free one, and a key moved
to a neighbouring voxel resolves to that voxel's index."""

import numpy as np

import oracle
import synth
from oracle.parity import frozen_from_device_keys, oracle_voxel_index


def test_frozen_from_own_keys_reproduces_the_gradient():
    cfg = synth.config1(seed=5, n_target=6000, n_source=2000)
    of = oracle.factor_from_clouds(cfg["sources"][0], cfg["targets"][0], cfg["resolutions"])
    pose = cfg["poses_true"][0]
    tr = of.linearize(pose, trace=True)
    found = np.where(tr["vidx"] >= 0, 1, 0).astype(np.int32)
    fz, n_face = frozen_from_device_keys(of, pose, tr["keys"], found)
    assert n_face == 0
    assert np.array_equal(fz, tr["vidx"])
    g0, gm0 = of.gradient(pose)
    g1, gm1 = of.gradient(pose, frozen=fz)
    np.testing.assert_array_equal(g0, g1)
    np.testing.assert_array_equal(gm0, gm1)


def test_voxel_index_lookup():
    cfg = synth.config1(seed=6, n_target=3000, n_source=10)
    vm = oracle.VoxelMap(cfg["targets"][0].xyz64(), cfg["targets"][0].cov64(), [0.5, 1.0])
    for level in (0, 1):
        keys = vm.levels[level][0]
        for v in (0, len(keys) // 2, len(keys) - 1):
            assert oracle_voxel_index(vm, level, keys[v]) == v
        assert oracle_voxel_index(vm, level, keys.max(axis=0) + 5) == -1
