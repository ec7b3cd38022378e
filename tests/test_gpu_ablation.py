"""Surface-validation ablation on the thin-wall scene, on the device: raw frames
preprocessed by the library, factors and Levenberg-Marquardt on the GPU
(needs an MI355X).  Same criteria as the oracle's ablation: without validation
the estimate started at the truth moves about one wall thickness across the
wall; with validation it stays within 2 cm."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

RES = [0.25, 0.5, 1.0]


@pytest.fixture(scope="module")
def vg():
    from paper_2407_10344_amd import vgicp
    ctx = vgicp.Context(0)
    yield vgicp, ctx
    ctx.close()


@pytest.mark.parametrize("seed", [1, 3])
def test_thin_wall_ablation_device(vg, seed):
    vgicp, ctx = vg
    d = synth.thin_wall_pair(seed)
    ct = vgicp.Cloud(ctx, d["target_raw"], 0.2, 10, np.zeros(3))
    cs = vgicp.Cloud(ctx, d["source_raw"], 0.2, 10, np.zeros(3))
    vm = vgicp.VoxelMap.from_cloud(ctx, ct, RES)
    src = vgicp.Source.from_cloud(ctx, cs)
    ct.close()
    cs.close()
    err = {}
    for validate in (False, True):
        batch = vgicp.FactorBatch(ctx, [src], [vm], viewpoints=np.zeros((1, 3)), precision="fp32c",
                                  validation=validate, use_graph=True)
        T = np.array([d["T_true"]])
        for _ in range(3):
            T, _, _ = batch.lm(T, iters=10)
        D = np.linalg.inv(d["T_true"]) @ T[0]
        err[validate] = float(np.linalg.norm(D[:3, 3]))
        batch.close()
    print("seed", seed, "translation error without / with validation:", err, flush=True)
    assert err[False] > 0.05
    assert err[True] < 0.02
    src.close()
    vm.close()
