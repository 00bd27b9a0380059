"""Occupancy integration of range scans on the GPU (edt_integrate_scan through
the C ABI) against the oracle: the occupancy after each scan bit for bit,
and the field, which must equal the oracle's transform of that occupancy."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2105_04419_amd import EDT_ERR_CAPACITY, EDT_ERR_RANGE, EdtError, Field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    oracle.build(force=False)


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).cuda()


def integrate(f, origin, ends, hits):
    return f.integrate_scan(dev(origin, np.int32), dev(ends, np.int32), dev(hits, np.uint8))


def check(f, occ, dmax, what):
    got = f.occupancy().cpu().numpy()
    if not np.array_equal(got, occ):
        bad = np.argwhere(got != occ)
        raise AssertionError(f"{what}: occupancy differs at {len(bad)} voxels, first {bad[0]}")
    assert np.array_equal(f.dense().cpu().numpy(), oracle.edt_separable(occ, dmax)), what


@pytest.mark.parametrize("seed", range(4))
def test_random_scans_on_boxes_map(seed):
    occ = workloads.dense_boxes(seed).copy()
    nz, ny, nx = occ.shape
    f = Field((nx, ny, nz), 20)
    f.global_(dev(occ, np.uint8))
    rng = np.random.default_rng(seed)
    for t in range(4):
        origin = np.array([rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)])
        n = 3000
        ends = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n), rng.integers(0, nz, n)], 1)
        hits = (rng.random(n) < 0.4).astype(np.uint8)
        integrate(f, origin, ends, hits)
        occ, skipped = oracle.integrate_scan(occ, origin, ends, hits)
        assert skipped == 0
        check(f, occ, 20, f"seed {seed} scan {t}")
    assert f.error() == 0


def test_single_rays_on_a_full_map():
    # every voxel occupied: a ray without a return clears exactly its walk
    nx, ny, nz = 40, 36, 30
    occ = np.ones((nz, ny, nx), np.uint8)
    f = Field((nx, ny, nz), 6)
    rng = np.random.default_rng(9)
    origin = np.array([20, 18, 15])
    ends = [[39, 18, 15], [0, 0, 0], [39, 35, 29], [25, 23, 20], [15, 13, 10], [20, 18, 15],
            [30, 23, 15], [12, 18, 19], [24, 26, 27]]
    ends += rng.integers(0, [nx, ny, nz], (20, 3)).tolist()
    for e in ends:
        f.global_(dev(occ, np.uint8))
        integrate(f, origin, np.array([e]), np.zeros(1, np.uint8))
        got = f.occupancy().cpu().numpy()
        freed = {tuple(v) for v in np.argwhere(got == 0)[:, ::-1]}
        assert freed == {tuple(v) for v in oracle.ray_voxels(origin, e)}, e
        # with a return, the end voxel stays occupied
        f.global_(dev(occ, np.uint8))
        integrate(f, origin, np.array([e]), np.ones(1, np.uint8))
        got = f.occupancy().cpu().numpy()
        freed_hit = {tuple(v) for v in np.argwhere(got == 0)[:, ::-1]}
        assert freed_hit == freed - {tuple(e)}, e


def test_tunnel_scans():
    from workloads.scans import ScanSim, tunnel_path
    occ = workloads.tunnels(0)
    nz, ny, nx = occ.shape
    xyz_b, data = workloads.dense_to_blocks(occ)
    f = Field((nx, ny, nz), 32)
    f.global_blocks(dev(xyz_b, np.int32), dev(data, np.uint8))
    sim = ScanSim(occ, tunnel_path(0), seed=0)
    cur = occ.copy()
    for t in range(3):
        pose, ends, hits = sim.rays()
        integrate(f, pose, ends, hits)
        cur, skipped = oracle.integrate_scan(cur, pose, ends, hits)
        assert skipped == 0
        check(f, cur, 32, f"tunnel scan {t}")
    assert f.error() == 0


def test_range_errors_and_capacity():
    occ = workloads.dense_boxes(1).copy()
    nz, ny, nx = occ.shape
    f = Field((nx, ny, nz), 10, max_changes=64)
    f.global_(dev(occ, np.uint8))
    with pytest.raises(EdtError) as e:
        integrate(f, [1, 1, 1], np.zeros((65, 3)), np.zeros(65))
    assert e.value.code == EDT_ERR_CAPACITY
    # origin outside: every ray skipped, nothing changes
    integrate(f, [-1, 5, 5], np.array([[3, 3, 3], [10, 10, 10]]), np.array([1, 0]))
    assert f.error() == EDT_ERR_RANGE
    check(f, occ, 10, "origin outside")
    # some rays outside: the others are integrated
    ends = np.array([[63, 40, 31], [64, 0, 0], [0, 63, 31], [5, 5, -2]])
    hits = np.array([1, 1, 0, 1], np.uint8)
    integrate(f, [32, 32, 16], ends, hits)
    assert f.error() == EDT_ERR_RANGE
    occ, skipped = oracle.integrate_scan(occ, [32, 32, 16], ends, hits)
    assert skipped == 2
    check(f, occ, 10, "rays outside")
    # too many voxels to free for the list: error, and the field still
    # matches whatever occupancy resulted
    full = np.ones((nz, ny, nx), np.uint8)
    f.global_(dev(full, np.uint8))
    rng = np.random.default_rng(2)
    ends = rng.integers(0, [nx, ny, nz], (40, 3))
    integrate(f, [32, 32, 16], ends, np.ones(40, np.uint8))
    assert f.error() == EDT_ERR_CAPACITY
    got = f.occupancy().cpu().numpy()
    assert (full - got).sum() <= 64 - 40
    assert np.array_equal(f.dense().cpu().numpy(), oracle.edt_separable(got, 10))
    for e in ends:                       # every hit end is occupied
        assert got[e[2], e[1], e[0]] == 1
