"""A block pool that grows (edt_grow; section IV-A: memory is allocated as
the transformed region grows).  An update that does not fit the pool is
cancelled with the map unchanged; after the pool grows (a copy of the pool
into a larger workspace, tile index rehashed), the same update gives the
oracle's field, and a grown field keeps its map, field, block count and
nearest obstacles exactly."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2105_04419_amd import Field
from test_gpu_nearest import all_voxels, check_nearest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    oracle.build(force=False)


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_full_pool_cancels_update_then_grow_and_repeat():
    nx, ny, nz = 96, 96, 40
    occ = np.zeros((nz, ny, nx), np.uint8)
    occ[4, 4, 4] = 1
    f = Field((nx, ny, nz), 8, max_blocks=12)
    f.global_(cu(occ))
    assert f.error() == 0
    before, occ_before = f.dense().cpu().numpy(), f.occupancy().cpu().numpy()
    xyz = np.array([[90, 90, 30], [5, 4, 4], [40, 60, 20]], np.int32)
    st = np.array([1, 1, 1], np.uint8)
    f.update(cu(xyz), cu(st))
    assert f.error() == -3                       # EDT_ERR_CAPACITY: cancelled
    assert np.array_equal(f.dense().cpu().numpy(), before), "a cancelled update changed s"
    assert np.array_equal(f.occupancy().cpu().numpy(), occ_before)
    f.grow(400)
    assert f.max_blocks == 400
    assert np.array_equal(f.dense().cpu().numpy(), before), "growth changed s"
    f.update(cu(xyz), cu(st))
    assert f.error() == 0
    occ[xyz[:, 2], xyz[:, 1], xyz[:, 0]] = 1
    assert np.array_equal(f.dense().cpu().numpy(), oracle.edt_separable(occ, 8))
    assert np.array_equal(f.occupancy().cpu().numpy(), occ)


def test_pool_full_in_the_first_kernel_leaves_the_map():
    # 4 free slots, 6 new blocks: the call is cancelled before any bit
    # changes (the case above fills the pool only during the dilation, after
    # the bits changed, and is rolled back)
    nx, ny, nz = 96, 96, 40
    occ = np.zeros((nz, ny, nx), np.uint8)
    occ[4, 4, 4] = 1
    f = Field((nx, ny, nz), 8, max_blocks=12)
    f.global_(cu(occ))
    before, occ_before = f.dense().cpu().numpy(), f.occupancy().cpu().numpy()
    xyz = np.array([[5, 4, 4]] + [[20 + 12 * i, 50, 30] for i in range(6)], np.int32)
    f.update(cu(xyz), cu(np.ones(len(xyz), np.uint8)))
    assert f.error() == -3
    assert np.array_equal(f.dense().cpu().numpy(), before)
    assert np.array_equal(f.occupancy().cpu().numpy(), occ_before)
    # the cancelled call left nothing behind that a fitting one would see
    near = np.array([[5, 4, 4], [4, 4, 4]], np.int32)
    f.update(cu(near), cu(np.array([1, 0], np.uint8)))
    assert f.error() == 0
    occ[4, 4, 5], occ[4, 4, 4] = 1, 0
    assert np.array_equal(f.dense().cpu().numpy(), oracle.edt_separable(occ, 8))
    assert np.array_equal(f.occupancy().cpu().numpy(), occ)


@pytest.mark.parametrize("dmax", [6, 20, 70])
def test_updates_grow_the_pool_on_demand(dmax):
    rng = np.random.default_rng(dmax)
    nx, ny, nz = 80, 72, 48
    occ = np.zeros((nz, ny, nx), np.uint8)
    occ[10:14, 10:12, 10:20] = 1
    f = Field((nx, ny, nz), dmax, max_blocks=8)
    f.global_(cu(occ), grow=True)
    assert np.array_equal(f.dense().cpu().numpy(), oracle.edt_separable(occ, dmax))
    first = f.max_blocks
    for step in range(6):
        n = 60
        xyz = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n),
                        rng.integers(0, nz, n)], 1).astype(np.int32)
        st = (rng.random(n) < 0.8).astype(np.uint8)
        for (x, y, z), v in zip(xyz, st):
            occ[z, y, x] = v
        f.update(cu(xyz), cu(st), grow=True)
        got = f.dense().cpu().numpy()
        assert np.array_equal(got, oracle.edt_separable(occ, dmax)), f"d={dmax} step {step}"
    # (at d_max 70 the first global already needs every block of the extent)
    assert f.max_blocks > first or first == f.extent_blocks
    g = Field((nx, ny, nz), dmax)
    g.global_(cu(occ))
    assert torch.equal(f.dense(), g.dense())
    # a grown field runs the global transform like a fresh one
    f.global_(cu(occ))
    assert torch.equal(f.dense(), g.dense())
    assert torch.equal(f.occupancy(), g.occupancy())


def test_grow_keeps_map_field_and_nearest_obstacles():
    occ = workloads.dense_boxes(3)
    nz, ny, nx = occ.shape
    f = Field((nx, ny, nz), 20, max_blocks=256)
    f.global_(cu(occ))
    rng = np.random.default_rng(5)
    xyz = np.stack([rng.integers(0, nx, 300), rng.integers(0, ny, 300),
                    rng.integers(0, nz, 300)], 1).astype(np.int32)
    st = (rng.random(300) < 0.5).astype(np.uint8)
    f.update(cu(xyz), cu(st))
    for (x, y, z), v in zip(xyz, st):
        occ[z, y, x] = v
    before = f.dense()
    blocks = f.stats()["blocks"]
    f.grow(256)                                  # same capacity: a move, not a resize
    f.grow()                                     # capped at the extent's blocks
    assert f.error() == 0
    assert torch.equal(f.dense(), before)
    assert f.stats()["blocks"] == blocks         # the pool is copied, not rebuilt
    ref = oracle.edt_separable(occ, 20)
    assert np.array_equal(before.cpu().numpy(), ref)
    q = all_voxels(nx, ny, nz)
    got = f.query_nearest(cu(q)).cpu().numpy()
    check_nearest(occ, ref.reshape(-1), q, got, 400, "nearest after growth")
    # and later updates still match the oracle
    f.update(cu(xyz[:50]), cu(1 - st[:50]))
    for (x, y, z), v in zip(xyz[:50], 1 - st[:50]):
        occ[z, y, x] = v
    assert np.array_equal(f.dense().cpu().numpy(), oracle.edt_separable(occ, 20))
