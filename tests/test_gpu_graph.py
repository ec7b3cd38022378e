"""Device two-node expansion and BSR assembly against the oracle's dense assembly
(needs an MI355X).  Per-factor expected values come from the oracle (with the
face-band rule), then oracle/graph.py assembles them; the device assembles its
own linearization.  Bar: relative 1e-5 (Frobenius) on the matrix and the rhs,
bitwise-identical repeated assemblies."""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.graph import assemble_dense
from oracle.parity import expected_with_device_keys, rel_err

pytestmark = pytest.mark.gpu


def test_graph_assembly_matches_oracle():
    from paper_2407_10344_amd import vgicp
    ctx = vgicp.Context(0)
    cfg = synth.config3(n_submaps=16, n_range=(15_000, 30_000), processes=4)
    maps, srcs, batch = vgicp.build_workload(ctx, cfg)
    poses = np.array(cfg["poses"])
    F = len(poses)
    d_poses = torch.tensor(vgicp.poses12(poses), device="cuda")
    lin, _ = batch.linearize_async(d_poses)
    node_i = [s for s, _ in cfg["factors"]]
    node_j = [t for _, t in cfg["factors"]]
    g = vgicp.Graph(ctx, 16, node_i, node_j)
    values, rhs = g.assemble(d_poses, lin)
    values2, rhs2 = g.assemble(d_poses, lin)
    torch.cuda.synchronize()
    assert torch.equal(values, values2) and torch.equal(rhs, rhs2)
    Hd_dev, bd_dev = g.dense(values, rhs)
    # expected per-factor terms from the oracle, then the oracle's assembly
    Hs, bs = [], []
    omaps = {}
    for f, (s, t) in enumerate(cfg["factors"]):
        if t not in omaps:
            tg = cfg["targets"][t]
            omaps[t] = oracle.VoxelMap(tg.xyz64(), tg.cov64(), cfg["resolutions"])
        src = cfg["sources"][s]
        of = oracle.Factor(src.xyz64(), src.cov64(), omaps[t])
        kd, fd = batch.correspondences(poses[f], f)
        e, H, b, _ = expected_with_device_keys(of, poses[f], kd, fd)
        Hs.append(H)
        bs.append(b)
    Hd, bd = assemble_dense(16, node_i, node_j, Hs, bs, list(poses))
    eH, eb = rel_err(Hd_dev, Hd), rel_err(bd_dev, bd)
    print("assembly rel err: H %.3g rhs %.3g, %d blocks" % (eH, eb, g.nnzb), flush=True)
    assert eH <= 1e-5 and eb <= 1e-5
    # structure: diagonal + both directions of every factor's node pair
    pairs = {(i, i) for i in range(16)} | {(i, j) for i, j in zip(node_i, node_j)} | {(j, i) for i, j in zip(node_i, node_j)}
    assert g.nnzb == len(pairs)
    g.close()
    batch.close()
    ctx.close()
