"""Nearest-obstacle query (the obst of a cell in Algorithm 1): several
obstacles can be equally near, so the tests compare what is unique (the
squared distance, against the oracle) and check that the returned voxel is
valid: inside the extent, occupied, and exactly that far away."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2105_04419_amd import Field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available()
    oracle.build(force=False)


def check_nearest(occ, ref, xyz, got, D, what):
    """occ (nz, ny, nx) uint8, ref: oracle s at the queries, xyz (n, 3) as
    (x, y, z), got (n, 3) nearest obstacles."""
    far = ref >= D
    assert (got[far] == -1).all(), f"{what}: a voxel without an obstacle within d_max got one"
    near = ~far
    o = got[near]
    q = xyz[near]
    nz, ny, nx = occ.shape
    inside = (o >= 0).all(1) & (o[:, 0] < nx) & (o[:, 1] < ny) & (o[:, 2] < nz)
    assert inside.all(), f"{what}: {int((~inside).sum())} answers outside the extent"
    assert (occ[o[:, 2], o[:, 1], o[:, 0]] != 0).all(), f"{what}: answer is not an obstacle"
    d2 = ((q - o).astype(np.int64) ** 2).sum(1)
    bad = np.nonzero(d2 != ref[near])[0]
    assert len(bad) == 0, (f"{what}: {len(bad)} answers at the wrong distance, first query "
                           f"{q[bad[0]]} -> {o[bad[0]]}: {d2[bad[0]]} vs {ref[near][bad[0]]}")


def all_voxels(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.int32)


@pytest.mark.parametrize("seed,dmax", [(0, 20), (1, 1), (2, 7), (3, 32), (4, 64), (5, 100)])
def test_every_voxel_of_boxes_map(seed, dmax):
    occ = workloads.dense_boxes(seed)
    nz, ny, nx = occ.shape
    f = Field((nx, ny, nz), dmax)
    f.global_(torch.from_numpy(occ).cuda())
    xyz = all_voxels(nx, ny, nz)
    got = f.query_nearest(torch.from_numpy(xyz).cuda()).cpu().numpy()
    ref = oracle.edt_separable(occ, dmax).reshape(-1)
    check_nearest(occ, ref, xyz, got, dmax * dmax, f"boxes seed {seed} d={dmax}")


def test_ragged_extent_and_out_of_extent_queries():
    rng = np.random.default_rng(8)
    occ = (rng.random((13, 21, 30)) < 0.01).astype(np.uint8)
    f = Field((30, 21, 13), 9)
    f.global_(torch.from_numpy(occ).cuda())
    xyz = all_voxels(30, 21, 13)
    got = f.query_nearest(torch.from_numpy(xyz).cuda()).cpu().numpy()
    check_nearest(occ, oracle.edt_separable(occ, 9).reshape(-1), xyz, got, 81, "ragged")
    out = np.array([[-1, 0, 0], [30, 0, 0], [0, 21, 0], [0, 0, 13]], np.int32)
    assert (f.query_nearest(torch.from_numpy(out).cuda()).cpu().numpy() == -1).all()


def test_tunnel_map_sample():
    occ = workloads.tunnels(0)
    nz, ny, nx = occ.shape
    xyz_b, data = workloads.dense_to_blocks(occ)
    f = Field((nx, ny, nz), 32)
    f.global_blocks(torch.from_numpy(xyz_b).cuda(), torch.from_numpy(data).cuda())
    rng = np.random.default_rng(1)
    # uniform voxels plus voxels near the walls
    walls = np.argwhere(occ)[rng.integers(0, int(occ.sum()), 100000)][:, ::-1]
    near = walls + rng.integers(-20, 21, walls.shape)
    xyz = np.concatenate([np.stack([rng.integers(0, nx, 100000), rng.integers(0, ny, 100000),
                                    rng.integers(0, nz, 100000)], 1), near])
    xyz = np.clip(xyz, 0, [nx - 1, ny - 1, nz - 1]).astype(np.int32)
    got = f.query_nearest(torch.from_numpy(xyz).cuda()).cpu().numpy()
    ref = oracle.edt_points(occ, 32, xyz)
    check_nearest(occ, ref, xyz, got, 1024, "tunnel")


@pytest.mark.parametrize("dmax", [20, 100])
def test_after_updates(dmax):
    # d_max 100 takes the envelope passes (radius beyond 64), whose pass Y
    # must leave the block minima the query reads for fresh and old blocks
    occ = workloads.dense_boxes(6)
    nz, ny, nx = occ.shape
    f = Field((nx, ny, nz), dmax)
    f.global_(torch.from_numpy(occ).cuda())
    rng = np.random.default_rng(2)
    xyz_all = all_voxels(nx, ny, nz)
    for step in range(6):
        n = 300
        xyz = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n), rng.integers(0, nz, n)],
                       1).astype(np.int32)
        st = (rng.random(n) < 0.5).astype(np.uint8)
        for (x, y, z), v in zip(xyz, st):
            occ[z, y, x] = v
        f.update(torch.from_numpy(xyz).cuda(), torch.from_numpy(st).cuda())
        got = f.query_nearest(torch.from_numpy(xyz_all).cuda()).cpu().numpy()
        check_nearest(occ, oracle.edt_separable(occ, dmax).reshape(-1), xyz_all, got,
                      dmax * dmax, f"after update {step} d={dmax}")
