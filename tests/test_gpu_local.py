"""Local-mapping batch (Sec. V-A): 15 raw frames preprocessed on the device,
matched all-to-all (105 factors) with surface validation on, against the FP64
oracle on its own preprocessing of the same raw frames (needs an MI355X)."""

import numpy as np
import pytest

import oracle
import synth
from oracle import preprocess as pp
from oracle.parity import check_factor

pytestmark = pytest.mark.gpu

RES = [0.25, 0.5, 1.0]


@pytest.fixture(scope="module")
def vg():
    from paper_2407_10344_amd import vgicp
    ctx = vgicp.Context(0)
    yield vgicp, ctx
    ctx.close()


def test_local_mapping_all_to_all(vg):
    vgicp, ctx = vg
    d = synth.local_mapping()
    N = len(d["raw"])
    clouds = [vgicp.Cloud(ctx, p, 0.25, 10, np.zeros(3)) for p in d["raw"]]
    srcs = [vgicp.Source.from_cloud(ctx, c) for c in clouds]
    maps = [vgicp.VoxelMap.from_cloud(ctx, c, RES) for c in clouds]
    for c in clouds:
        c.close()
    pairs = d["pairs"]
    batch = vgicp.FactorBatch(ctx, [srcs[i] for i, _ in pairs], [maps[j] for _, j in pairs],
                              viewpoints=np.zeros((len(pairs), 3)), precision="fp32c", validation=True,
                              use_graph=True)
    poses = np.array(d["rel_est"])
    e, H, b, inl = batch.linearize(poses)
    e2, H2, b2, _ = batch.linearize(poses)
    assert np.array_equal(e, e2) and np.array_equal(H, H2) and np.array_equal(b, b2)
    print("frames", N, "factors", len(pairs), "inliers per level (mean)", inl.mean(axis=0).round(1), flush=True)
    ops = [pp.preprocess(p, 0.25, 10, np.zeros(3), search="tree") for p in d["raw"]]
    omaps = [oracle.VoxelMap(o["xyz"], pp.cov6(o["cov"]), RES) for o in ops]
    worst = {"e": 0.0, "H": 0.0, "b": 0.0}
    for f, (i, j) in enumerate(pairs):
        ofac = oracle.Factor(ops[i]["xyz"], pp.cov6(ops[i]["cov"]), omaps[j], nrm=ops[i]["normals"],
                             viewpoint=np.zeros(3), validate=True)
        errs, _ = check_factor(batch, f, poses[f], ofac, e[f], H[f], b[f])
        worst = {k: max(worst[k], errs[k]) for k in worst}
    print("worst relative errors over all factors", worst, flush=True)
    batch.close()
    for x in srcs + maps:
        x.close()
