"""Full (uncapped) transform of dense grids on the GPU (edt_dense_global
through the C ABI) against the oracle, bit for bit: boxes maps, ragged
random grids, long rows with values far beyond 16 bits, capped radii beyond
the sparse field's 255, the empty and full grids, sampled voxels of the full
tunnel extent, and argument errors."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2105_04419_amd import DENSE_INF, EDT_ERR_ARG, EdtError, Field, dense_global, lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    oracle.build(force=False)


def run(occ, d_max=0):
    return dense_global(torch.from_numpy(np.ascontiguousarray(occ)).cuda(), d_max).cpu().numpy()


def same(got, ref, what):
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        z, y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} mismatches, first at x={x} y={y} z={z}: "
                             f"gpu={got[z, y, x]} oracle={ref[z, y, x]}")


@pytest.mark.parametrize("seed", range(5))
def test_boxes_uncapped_and_capped(seed):
    occ = workloads.dense_boxes(seed)
    same(run(occ), oracle.edt_uncapped(occ), f"boxes {seed} uncapped")
    capped = run(occ, 20)
    same(capped, oracle.edt_separable(occ, 20), f"boxes {seed} d=20")
    # the sparse field agrees
    nz, ny, nx = occ.shape
    f = Field((nx, ny, nz), 20)
    f.global_(torch.from_numpy(occ).cuda())
    assert np.array_equal(f.dense().cpu().numpy(), capped)


@pytest.mark.parametrize("shape,p", [
    ((45, 33, 70), 0.01), ((7, 5, 130), 0.05), ((200, 1, 1), 0.02), ((1, 200, 1), 0.02),
    ((1, 1, 200), 0.02), ((30, 29, 65), 0.0005), ((3, 64, 64), 0.5), ((17, 19, 23), 1.0),
    ((1, 1, 1), 1.0), ((2, 3, 129), 0.001),
])
def test_ragged_random(shape, p):
    rng = np.random.default_rng(int(p * 1e4) + sum(shape))
    occ = (rng.random(shape) < p).astype(np.uint8)
    if not occ.any():
        occ.reshape(-1)[rng.integers(0, occ.size)] = 1
    same(run(occ), oracle.edt_uncapped(occ), f"{shape} p={p}")


def test_long_rows_beyond_16_bits():
    for axis in range(3):
        shape = [3, 3, 3]
        shape[axis] = 700
        occ = np.zeros(shape, np.uint8)
        idx = [1, 1, 1]
        idx[axis] = 0
        occ[tuple(idx)] = 1
        got = run(occ)
        same(got, oracle.edt_uncapped(occ), f"long axis {axis}")
        assert got.max() == 699 ** 2 + 2


@pytest.mark.parametrize("d_max", [1, 300, 1000])
def test_large_radii(d_max):
    rng = np.random.default_rng(d_max)
    occ = (rng.random((40, 50, 300)) < 0.0002).astype(np.uint8)
    occ[0, 0, 0] = 1
    same(run(occ, d_max), oracle.edt_separable(occ, d_max), f"d_max {d_max}")


def test_empty_and_full():
    assert (run(np.zeros((9, 10, 70), np.uint8)) == DENSE_INF).all()
    assert (run(np.zeros((9, 10, 70), np.uint8), 12) == 144).all()
    assert (run(np.ones((9, 10, 70), np.uint8)) == 0).all()


def test_tunnel_extent_sampled():
    occ = workloads.tunnels(0)
    nz, ny, nx = occ.shape
    got = run(occ)
    rng = np.random.default_rng(7)
    q = np.stack([rng.integers(0, nx, 600), rng.integers(0, ny, 600), rng.integers(0, nz, 600)], 1)
    obs = np.argwhere(occ)[:, ::-1]
    want = oracle.edt_points_list(obs, 46340, q)
    assert np.array_equal(got[q[:, 2], q[:, 1], q[:, 0]], want)
    # capped at 32 it equals the oracle's field everywhere
    same(np.minimum(got, 1024), oracle.edt_separable(occ, 32), "tunnel min(D, uncapped)")


def test_argument_errors():
    L = lib()
    assert L.edt_dense_workspace_bytes(46341, 1, 1) == EDT_ERR_ARG
    assert L.edt_dense_workspace_bytes(0, 4, 4) == EDT_ERR_ARG
    occ = torch.zeros((4, 4, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(EdtError):
        dense_global(occ, -1)
    with pytest.raises(EdtError):
        dense_global(occ, 46341)


def test_largest_extent_squared_distances_near_int32_max():
    # nx^2 + ny^2 + nz^2 just below 2^31: one obstacle in a corner gives
    # squared distances up to 46338^2 + 2, exact in int32
    nx, ny, nz = 46339, 2, 2
    occ = np.zeros((nz, ny, nx), np.uint8)
    occ[0, 0, 0] = 1
    got = run(occ)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    want = x.astype(np.int64) ** 2 + y ** 2 + z ** 2
    assert np.array_equal(got.astype(np.int64), want)
    assert int(got.max()) == 46338 ** 2 + 2
    # and capped at the largest radius
    assert np.array_equal(run(occ, 46340).astype(np.int64), np.minimum(want, 46340 ** 2))
