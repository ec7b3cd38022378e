"""The allocation-free linearization (vg_linearize_noalloc) through the C ABI
(needs an MI355X): the same results as vg_linearize_async, bit for bit, on two
calls in a row (the second with a smaller batch, so the fixed scratch holds the
first call's rows), and a clear error for a batch beyond the fixed scratch."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    from paper_2407_10344_amd import vgicp
    ctx = vgicp.Context(0)
    yield vgicp, ctx
    ctx.close()


def _both(batch, d_poses):
    out_a, inl_a = batch.linearize_async(d_poses)
    out_n = torch.full_like(out_a, float("nan"))
    inl_n = torch.full_like(inl_a, -1)
    batch.linearize_noalloc(d_poses, out_n, inl_n)
    torch.cuda.synchronize()
    return out_a.cpu().numpy(), inl_a.cpu().numpy(), out_n.cpu().numpy(), inl_n.cpu().numpy()


def test_noalloc_matches_async_on_two_calls(vg):
    vgicp, ctx = vg
    big = synth.config2(seed=2)                     # 20 factors x ~32k points, 4 levels
    small = synth.config1(seed=1)                   # 1 factor, 5k points
    _, _, b_big = vgicp.build_workload(ctx, big)
    _, _, b_small = vgicp.build_workload(ctx, small)
    for name, batch, cfg in (("odometry", b_big, big), ("single", b_small, small), ("odometry", b_big, big)):
        d_poses = torch.tensor(vgicp.poses12(np.array(cfg["poses"])), device="cuda")
        oa, ia, on, inn = _both(batch, d_poses)
        print(name, "tiles", batch.info()["n_tiles"], "e", oa[:2, 0].tolist(), flush=True)
        assert np.array_equal(oa, on) and np.array_equal(ia, inn)
        # and the host-buffer entry point agrees too
        e, H, b, inl = batch.linearize(cfg["poses"])
        assert np.array_equal(on[:, 0], e) and np.array_equal(on[:, 1:37].reshape(-1, 6, 6), H)
        assert np.array_equal(on[:, 37:], b) and np.array_equal(inn, inl)
    b_big.close()
    b_small.close()


def test_noalloc_refuses_batches_beyond_its_scratch(vg):
    from paper_2407_10344_amd._lib import VGError
    vgicp, ctx = vg
    c = synth.config1(seed=3, n_target=5000, n_source=70_000)
    maps, srcs, _ = vgicp.build_workload(ctx, c)
    src, m = srcs[0], maps[0]
    batch = vgicp.FactorBatch(ctx, [src] * 100, [m] * 100, tile=64, block=64)    # ~110k tiles
    assert batch.info()["n_tiles"] > 105_000
    d_poses = torch.tensor(vgicp.poses12([c["poses_true"][0]] * 100), device="cuda")
    out = torch.empty((100, 43), dtype=torch.float64, device="cuda")
    with pytest.raises(VGError, match="CAPACITY.*fixed scratch"):
        batch.linearize_noalloc(d_poses, out)
    batch.close()
