"""Voxel-map edge cases on the device (needs an MI355X), against the FP64 oracle:
many points in one voxel, block-table probe chains forced by colliding slots,
and the per-level voxel capacity (Sec. III-C, Preprocessing and Correspondence
search)."""

import numpy as np
import pytest

import oracle
from oracle.parity import check_factor

pytestmark = pytest.mark.gpu

GOLDEN = 0x9E3779B1


@pytest.fixture(scope="module")
def vg():
    from paper_2407_10344_amd import vgicp
    ctx = vgicp.Context(0)
    yield vgicp, ctx
    ctx.close()


def _covs(rng, n, scale=0.1):
    A = rng.normal(size=(n, 3, 3)) * scale
    C = A @ np.transpose(A, (0, 2, 1)) + 0.01 * np.eye(3)
    return np.stack([C[:, 0, 0], C[:, 0, 1], C[:, 0, 2], C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]], 1)


def slot_of_block(b, log2cap):
    """Slot of a block in the device table (white box: the map build's hash): the
    block key packs the voxel key + 8192, shifted right by 2, 12 bits per axis,
    x highest; its two 32-bit words are XORed and Fibonacci-hashed."""
    bx, by, bz = ((4 * int(v) + 8192) >> 2 for v in b)
    bk = (bx << 24) | (by << 12) | bz
    w = ((bk & 0xFFFFFFFF) ^ (bk >> 32)) & 0xFFFFFFFF
    return ((w * GOLDEN) & 0xFFFFFFFF) >> (32 - log2cap)


def test_many_points_in_one_voxel(vg):
    """200,000 points in one voxel and a few hundred elsewhere: keys, counts, means
    and covariances bit-exact against the oracle, and a factor linearized into
    the map matches it."""
    vgicp, ctx = vg
    rng = np.random.default_rng(5)
    r = 0.5
    heavy = np.array([1.75, 1.75, 1.75]) + rng.uniform(-0.2, 0.2, size=(200_000, 3))
    rest = rng.uniform(-4.0, 4.0, size=(400, 3))
    xyz = np.concatenate([[[0.1, 0.1, 0.1]], heavy, rest])
    cov = _covs(rng, xyz.shape[0])
    m = vgicp.VoxelMap(ctx, xyz, cov, [r])
    k_o, m_o, c_o, n_o = oracle.voxelize(xyz, cov, r)
    k_d, m_d, c_d, n_d = m.export(0)
    assert np.array_equal(k_d, k_o) and np.array_equal(n_d, n_o)
    assert n_o.max() >= 200_000
    assert np.array_equal(m_d, m_o) and np.array_equal(c_d, c_o)
    src = np.concatenate([heavy[:5000] + rng.normal(scale=0.01, size=(5000, 3)),
                          rest + rng.normal(scale=0.01, size=rest.shape)])
    scov = _covs(rng, src.shape[0])
    s = vgicp.Source(ctx, src, scov)
    of = oracle.Factor(src, scov, oracle.VoxelMap(xyz, cov, [r]))
    pose = np.eye(4)
    pose[:3, 3] = [0.003, -0.002, 0.001]
    for prec in ("fp32c", "fp64"):
        batch = vgicp.FactorBatch(ctx, [s], [m], precision=prec)
        e, H, b, inl = batch.linearize([pose])
        assert inl[0, 0] == of.linearize(pose)["inliers"][0]
        check_factor(batch, 0, pose, of, e[0], H[0], b[0])
        batch.close()
    s.close()
    m.close()


def test_colliding_blocks_walk_the_probe_chain(vg):
    """Twelve occupied blocks whose table slots coincide (one chain of twelve
    entries in a 64-slot table) and five more absent ones on the same slot:
    occupied voxels are found, empty voxels of occupied blocks and voxels of the
    absent blocks (whose lookup walks the whole chain to an empty slot) are not;
    keys and found flags equal the oracle's in both precision modes, and so do
    e, H and b."""
    vgicp, ctx = vg
    rng = np.random.default_rng(8)
    r = 1.0
    lg = 6                                    # 64 slots: 4 x (12 blocks) <= 64
    origin_block = (0, 0, 0)
    s0 = slot_of_block(origin_block, lg)
    cands = [(x, y, z) for x in range(-6, 7) for y in range(-6, 7) for z in range(-6, 7)
             if (x, y, z) != origin_block and slot_of_block((x, y, z), lg) == s0]
    rng.shuffle(cands)
    assert len(cands) >= 16
    occupied = [origin_block] + [tuple(c) for c in cands[:11]]
    absent = [tuple(c) for c in cands[11:16]]

    def in_voxel(block, local, jitter=0.3, n=1):
        v = np.array(block) * 4 + np.array(local)
        return v + 0.5 + rng.uniform(-jitter, jitter, size=(n, 3))

    tgt, used = [np.array([[0.5, 0.5, 0.5]])], {}
    for blk in occupied:
        locs = {tuple(rng.integers(0, 4, size=3)) for _ in range(3)}
        if blk == origin_block:
            locs.add((0, 0, 0))
        used[blk] = locs
        for loc in locs:
            tgt.append(in_voxel(blk, loc, n=int(rng.integers(1, 20))))
    xyz = np.concatenate(tgt)
    cov = _covs(rng, xyz.shape[0])
    m = vgicp.VoxelMap(ctx, xyz, cov, [r])
    V, cap = m.info(0)
    assert cap == 1 << lg and V == sum(len(v) for v in used.values())

    src = []
    for blk, locs in used.items():
        for loc in locs:
            src.append(in_voxel(blk, loc, jitter=0.2))                        # found
        free = [(x, y, z) for x in range(4) for y in range(4) for z in range(4) if (x, y, z) not in locs]
        for k in rng.choice(len(free), size=3, replace=False):
            src.append(in_voxel(blk, free[k], jitter=0.2))                    # empty voxel of the block
    lo, hi = np.floor(xyz.min(0)), np.floor(xyz.max(0))
    for blk in absent:
        for _ in range(3):
            p = in_voxel(blk, tuple(rng.integers(0, 4, size=3)), jitter=0.2)
            if np.all((np.floor(p) >= lo) & (np.floor(p) <= hi)):         # inside the key box: probed
                src.append(p)
    src = np.concatenate(src)
    scov = _covs(rng, src.shape[0])
    s = vgicp.Source(ctx, src, scov)
    of = oracle.Factor(src, scov, oracle.VoxelMap(xyz, cov, [r]))
    pose = np.eye(4)
    tr = of.linearize(pose, trace=True)
    n_absent = sum(1 for p in np.floor(src).astype(int) if tuple(p // 4) in set(absent))
    assert n_absent >= 3 and (tr["vidx"][:, 0] >= 0).sum() == V
    for prec in ("fp32c", "fp64"):
        batch = vgicp.FactorBatch(ctx, [s], [m], precision=prec)
        keys_d, found_d = batch.correspondences(pose, 0)
        assert np.array_equal(keys_d[:, 0], tr["keys"][:, 0])
        assert np.array_equal(found_d[:, 0] == 1, tr["vidx"][:, 0] >= 0)
        e, H, b, inl = batch.linearize([pose])
        assert inl[0, 0] == V
        check_factor(batch, 0, pose, of, e[0], H[0], b[0])
        batch.close()
    s.close()
    m.close()


def test_voxel_capacity_per_level(vg):
    """A level holds at most 2^26 - 1 voxels (64-byte records addressed by 32-bit
    byte offsets): a one-voxel-per-point lattice of 2^26 - 1 points builds, one
    more point is refused with VG_ERR_CAPACITY."""
    vgicp, ctx = vg
    from paper_2407_10344_amd._lib import VGError
    side = 8192
    n = side * side                                    # 2^26
    g = (np.arange(side, dtype=np.float64) - side // 2) + 0.5
    xyz = np.empty((n, 3))
    xyz[:, 0] = np.repeat(g, side)
    xyz[:, 1] = np.tile(g, side)
    xyz[:, 2] = 0.5
    i0 = side * (side // 2) + side // 2                # the point at (0.5, 0.5, 0.5) goes first: map origin 0
    xyz[[0, i0]] = xyz[[i0, 0]]
    cov = np.empty((n, 6))
    cov[:] = [0.01, 0.0, 0.0, 0.01, 0.0, 0.01]
    print("building %d-voxel level" % (n - 1), flush=True)
    m = vgicp.VoxelMap(ctx, xyz[: n - 1], cov[: n - 1], [1.0])
    V, cap = m.info(0)
    assert V == n - 1
    m.close()
    print("building %d-voxel level" % n, flush=True)
    with pytest.raises(VGError) as ei:
        vgicp.VoxelMap(ctx, xyz, cov, [1.0])
    assert ei.value.status == -5
