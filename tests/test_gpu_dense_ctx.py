"""Incremental uncapped transform of dense grids (edt_dense_ctx_* through the
C ABI): after every update the field equals the oracle's field of the new
occupancy bit for bit (uncapped and capped beyond the sparse field's radii),
with duplicates (last entry wins), no-op entries, removal of every obstacle,
rows longer than one 1024-voxel chunk, argument and range errors, and range
scans on the full tunnel extent checked against the global dense transform
and sampled voxels of the definition."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from workloads.scans import ScanSim, tunnel_path
from paper_2105_04419_amd import (DENSE_INF, EDT_ERR_ARG, EDT_ERR_CAPACITY, EDT_ERR_RANGE,
                                  DenseField, EdtError, dense_global, lib)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    oracle.build(force=False)


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ref(occ, d_max):
    return oracle.edt_uncapped(occ) if d_max == 0 else oracle.edt_separable(occ, d_max)


def same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        z, y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} mismatches, first at x={x} y={y} z={z}: "
                             f"gpu={got[z, y, x]} oracle={want[z, y, x]}")


def random_changes(rng, occ, n, p_add):
    nz, ny, nx = occ.shape
    xyz = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n), rng.integers(0, nz, n)],
                   1).astype(np.int32)
    st = (rng.random(n) < p_add).astype(np.uint8)
    return xyz, st


def apply(occ, xyz, st):
    for (x, y, z), v in zip(xyz, st):          # in order: the last entry wins
        occ[z, y, x] = v


@pytest.mark.parametrize("shape,d_max", [
    ((45, 33, 70), 0), ((7, 5, 130), 0), ((64, 64, 32), 0), ((30, 29, 65), 300),
    ((1100, 3, 2), 0), ((2, 3, 129), 0), ((17, 19, 23), 5),
])
def test_updates_match_the_oracle(shape, d_max):
    nx, ny, nz = shape
    rng = np.random.default_rng(nx * 7 + ny * 3 + nz + d_max)
    occ = (rng.random((nz, ny, nx)) < 0.01).astype(np.uint8)
    f = DenseField(shape, d_max, max_changes=256)
    f.global_(cu(occ))
    same(f.field().cpu().numpy(), ref(occ, d_max), f"{shape} global")
    for step in range(8):
        n = int(rng.integers(1, 120))
        xyz, st = random_changes(rng, occ, n, 0.6 if step % 2 == 0 else 0.3)
        if step == 3:                          # duplicates with different states
            xyz = np.concatenate([xyz, xyz[:10]])
            st = np.concatenate([st, 1 - st[:10]])
        f.update(cu(xyz), cu(st))
        apply(occ, xyz, st)
        same(f.field().cpu().numpy(), ref(occ, d_max), f"{shape} d={d_max} step {step}")
    assert f.error() == 0


def test_remove_every_obstacle_then_add_one():
    nx, ny, nz = 40, 30, 20
    occ = np.zeros((nz, ny, nx), np.uint8)
    occ[3, 4, 5] = occ[10, 20, 30] = occ[19, 29, 39] = 1
    f = DenseField((nx, ny, nz), 0, max_changes=16)
    f.global_(cu(occ))
    obs = np.argwhere(occ)[:, ::-1].astype(np.int32)
    f.update(cu(obs), cu(np.zeros(len(obs), np.uint8)))
    assert (f.field().cpu().numpy() == DENSE_INF).all()
    f.update(cu(np.array([[0, 0, 0]], np.int32)), cu(np.array([1], np.uint8)))
    occ[:] = 0
    occ[0, 0, 0] = 1
    same(f.field().cpu().numpy(), oracle.edt_uncapped(occ), "single obstacle after emptying")


def test_noop_entries_change_nothing():
    occ = workloads.dense_boxes(2)
    nz, ny, nx = occ.shape
    f = DenseField((nx, ny, nz), 0, max_changes=512)
    f.global_(cu(occ))
    before = f.field().clone()
    xyz = np.argwhere(occ)[:200, ::-1].astype(np.int32)
    f.update(cu(xyz), cu(np.ones(len(xyz), np.uint8)))       # already occupied
    free = np.argwhere(occ == 0)[:200, ::-1].astype(np.int32)
    f.update(cu(free), cu(np.zeros(len(free), np.uint8)))    # already free
    assert torch.equal(f.field(), before)
    # set and clear in one call: the last entry wins, nothing changes
    f.update(cu(np.concatenate([free[:5], free[:5]])),
             cu(np.array([1] * 5 + [0] * 5, np.uint8)))
    assert torch.equal(f.field(), before)


def test_range_error_cancels_the_call_and_capacity():
    occ = workloads.dense_boxes(1)
    nz, ny, nx = occ.shape
    f = DenseField((nx, ny, nz), 0, max_changes=8)
    f.global_(cu(occ))
    before = f.field().clone()
    xyz = np.array([[1, 1, 1], [nx, 0, 0]], np.int32)
    f.update(cu(xyz), cu(np.array([1, 1], np.uint8)))
    assert f.error() == EDT_ERR_RANGE
    assert torch.equal(f.field(), before)
    assert f.error() == 0                                      # reading clears it
    with pytest.raises(EdtError) as e:
        f.update(cu(np.zeros((9, 3), np.int32)), cu(np.ones(9, np.uint8)))
    assert e.value.code == EDT_ERR_CAPACITY
    L = lib()
    assert L.edt_dense_ctx_bytes(0, 4, 4, 8) == EDT_ERR_ARG
    assert L.edt_dense_ctx_bytes(4, 4, 4, 0) == EDT_ERR_ARG
    with pytest.raises(EdtError):
        DenseField((4, 4, 4), 46341)


def test_tunnel_scans_full_extent():
    occ = workloads.tunnels(0)
    nz, ny, nx = occ.shape
    sim = ScanSim(occ, tunnel_path(0), seed=0)
    f = DenseField((nx, ny, nz), 0, max_changes=1 << 16)
    f.global_(cu(occ))
    rng = np.random.default_rng(3)
    for scan in range(12):
        xyz, st = sim.step()[:2]
        f.update(cu(xyz), cu(st))
        cur = sim.map
        if scan % 4 == 3:
            g = dense_global(cu(cur))
            assert torch.equal(f.field(), g), f"scan {scan}: incremental != global"
            q = np.stack([rng.integers(0, nx, 300), rng.integers(0, ny, 300),
                          rng.integers(0, nz, 300)], 1)
            obs = np.argwhere(cur)[:, ::-1]
            got = f.field().cpu().numpy()[q[:, 2], q[:, 1], q[:, 0]]
            assert np.array_equal(got, oracle.edt_points_list(obs, 46340, q)), f"scan {scan}"
    assert f.error() == 0
