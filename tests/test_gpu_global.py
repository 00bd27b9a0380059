"""Global transform on the GPU (libedt through its C ABI) against the CPU
oracle, bit for bit: dense 64x64x32 boxes maps, tiny adversarial grids, the
leaf-block input form, and the full 1024x1024x128 tunnel map."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2105_04419_amd import Field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    oracle.build(force=False)


def gpu_field(occ, dmax, **kw):
    nz, ny, nx = occ.shape
    f = Field((nx, ny, nz), dmax, **kw)
    f.global_(torch.from_numpy(np.ascontiguousarray(occ)).cuda())
    return f


def assert_same(got, ref, what=""):
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        z, y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} mismatches, first at x={x} y={y} z={z}: "
                             f"gpu={got[z, y, x]} oracle={ref[z, y, x]}")


@pytest.mark.parametrize("seed", range(10))
def test_dense_boxes_matches_oracle(seed):
    occ = workloads.dense_boxes(seed)
    f = gpu_field(occ, 20)
    got = f.dense().cpu().numpy()
    assert_same(got, oracle.edt_separable(occ, 20), f"dense_boxes seed {seed}")
    assert f.error() == 0


@pytest.mark.parametrize("shape,p,dmax", [
    ((1, 1, 1), 0.0, 1), ((1, 1, 1), 1.0, 3), ((5, 7, 13), 0.05, 2),
    ((3, 17, 9), 0.02, 8), ((40, 3, 100), 0.003, 20), ((33, 31, 29), 0.001, 32),
    ((16, 16, 16), 0.0005, 255), ((24, 40, 72), 0.0002, 255), ((9, 9, 9), 0.3, 1),
    ((64, 8, 8), 0.01, 12), ((8, 64, 8), 0.01, 12), ((8, 8, 64), 0.01, 12),
    ((17, 130, 19), 0.002, 40), ((130, 17, 19), 0.002, 40),
    # window radii M = 6, 7, 8 and the first radius of the envelope path, on
    # extents spanning several 64-voxel tiles along every pass axis
    ((66, 70, 140), 0.0008, 48), ((140, 66, 70), 0.0008, 56),
    ((72, 150, 80), 0.0004, 64), ((150, 72, 80), 0.0004, 57),
    ((80, 80, 80), 0.0003, 65), ((70, 140, 66), 0.0006, 100),
])
def test_adversarial_grids(shape, p, dmax):
    rng = np.random.default_rng(hash((shape, p, dmax)) % (1 << 32))
    occ = (rng.random(shape) < p).astype(np.uint8)
    # obstacles on faces, edges and corners
    nz, ny, nx = shape
    occ[0, 0, 0] = 1 if p > 0 else 0
    if p > 0:
        occ[nz - 1, ny - 1, nx - 1] = 1
        occ[nz // 2, 0, nx - 1] = 1
    f = gpu_field(occ, dmax)
    assert_same(f.dense().cpu().numpy(), oracle.edt_bruteforce(occ, dmax), f"{shape} d={dmax}")


def test_empty_and_full():
    occ = np.zeros((20, 30, 40), np.uint8)
    f = gpu_field(occ, 7)
    assert (f.dense().cpu().numpy() == 49).all()
    assert f.stats()["blocks"] == 0
    f.global_(torch.ones((20, 30, 40), dtype=torch.uint8, device="cuda"))
    assert (f.dense().cpu().numpy() == 0).all()


def test_values_as_occupancy():
    """Any nonzero byte is an obstacle."""
    occ = workloads.dense_boxes(3)
    occ2 = occ * np.uint8(173)
    f = gpu_field(occ2, 20)
    assert_same(f.dense().cpu().numpy(), oracle.edt_separable(occ, 20))
    assert np.array_equal(f.occupancy().cpu().numpy(), (occ != 0).astype(np.uint8))


def test_block_input_equals_dense_input():
    occ = workloads.dense_boxes(4)
    xyz, data = workloads.dense_to_blocks(occ)
    f = Field((64, 64, 32), 20)
    f.global_blocks(torch.from_numpy(xyz).cuda(), torch.from_numpy(data).cuda())
    assert_same(f.dense().cpu().numpy(), oracle.edt_separable(occ, 20))
    # repeated blocks merge by union
    half = data.copy()
    half[:, ::2] = 0
    xyz2 = np.concatenate([xyz, xyz])
    data2 = np.concatenate([half, data - half])
    f.global_blocks(torch.from_numpy(xyz2).cuda(), torch.from_numpy(data2).cuda())
    assert_same(f.dense().cpu().numpy(), oracle.edt_separable(occ, 20))


def test_block_input_repeats_beyond_pool_size():
    """More repeated listings than pool slots: every listing is still merged
    (the repeat list overflows and all blocks are ORed in again)."""
    rng = np.random.default_rng(11)
    occ = np.zeros((16, 16, 16), np.uint8)
    occ[4:12, 4:12, 4:12] = (rng.random((8, 8, 8)) < 0.3)
    xyz, data = workloads.dense_to_blocks(occ)
    # each voxel of each block goes to one of 40 listings of that block
    pick = rng.integers(0, 40, size=data.shape)
    xyz_r = np.concatenate([xyz] * 40)
    data_r = np.concatenate([np.where(pick == k, data, 0) for k in range(40)]).astype(np.uint8)
    f = Field((16, 16, 16), 5, max_blocks=8)
    assert len(xyz_r) - len(xyz) > 8
    f.global_blocks(torch.from_numpy(xyz_r).cuda(), torch.from_numpy(data_r).cuda())
    assert f.error() == 0
    assert_same(f.dense().cpu().numpy(), oracle.edt_separable(occ, 5))


def test_tile_created_as_neighbour_then_obstacle():
    """A tile first created as the neighbour of an obstacle tile and only then
    given an obstacle block must still bring its own neighbourhood into the
    region.  Tile x = 0 holds an obstacle deep inside, tile x = 1 one on its
    +x face, tile x = 2 none but voxels within d_max of the second obstacle.
    The block list puts the first obstacle at entry 0 and the second at entry
    131072 with empty blocks between: the ingest walks its input with at most
    16384 waves of 8 blocks, so one wave takes both, in that order, and tile
    x = 1 already exists (as a neighbour) when its obstacle arrives."""
    nx, ny, nz = 192, 64, 64
    occ = np.zeros((nz, ny, nx), np.uint8)
    occ[32, 32, 10] = 1
    occ[32, 32, 127] = 1
    ref = oracle.edt_separable(occ, 32)
    xyz, data = workloads.dense_to_blocks(occ)
    a = int(np.argmin(xyz[:, 0]))
    b = int(np.argmax(xyz[:, 0]))
    n = 16384 * 8 + 1
    xyz_l = np.zeros((n, 3), np.int32)                 # empty blocks at the origin
    data_l = np.zeros((n, 512), np.uint8)
    xyz_l[0], data_l[0] = xyz[a], data[a]
    xyz_l[n - 1], data_l[n - 1] = xyz[b], data[b]
    f = Field((nx, ny, nz), 32)
    f.global_blocks(torch.from_numpy(xyz_l).cuda(), torch.from_numpy(data_l).cuda())
    assert f.error() == 0
    assert_same(f.dense().cpu().numpy(), ref, "block input")
    f.global_(torch.from_numpy(occ).cuda())
    assert_same(f.dense().cpu().numpy(), ref, "dense input")


def test_block_input_ragged_extent_and_range_error():
    """Voxels of a block beyond the extent are ignored; blocks outside the
    extent are skipped and reported."""
    nx, ny, nz = 21, 13, 10
    rng = np.random.default_rng(5)
    full = (rng.random((16, 16, 24)) < 0.02).astype(np.uint8)
    xyz, data = workloads.dense_to_blocks(full)
    f = Field((nx, ny, nz), 6)
    f.global_blocks(torch.from_numpy(xyz).cuda(), torch.from_numpy(data).cuda())
    assert f.error() == 0
    assert_same(f.dense().cpu().numpy(), oracle.edt_bruteforce(full[:nz, :ny, :nx], 6))
    bad = np.array([[5, 0, 0]], np.int32)
    f.global_blocks(torch.from_numpy(bad).cuda(), torch.ones((1, 512), dtype=torch.uint8).cuda())
    assert f.error() == -2
    assert (f.dense().cpu().numpy() == 36).all()


def test_query_matches_dense_and_background():
    occ = workloads.dense_boxes(5)
    f = gpu_field(occ, 20)
    ref = oracle.edt_separable(occ, 20)
    rng = np.random.default_rng(0)
    xyz = np.stack([rng.integers(-5, 70, 4000), rng.integers(-5, 70, 4000),
                    rng.integers(-5, 40, 4000)], 1).astype(np.int32)
    got = f.query(torch.from_numpy(xyz).cuda()).cpu().numpy()
    inside = (xyz[:, 0] < 64) & (xyz[:, 1] < 64) & (xyz[:, 2] < 32) & (xyz >= 0).all(1)
    exp = np.full(len(xyz), 400, np.int32)
    exp[inside] = ref[xyz[inside, 2], xyz[inside, 1], xyz[inside, 0]]
    assert np.array_equal(got, exp)


def test_deterministic_rerun():
    occ = workloads.dense_boxes(6)
    f = gpu_field(occ, 20)
    a = f.dense().cpu().numpy()
    f.global_(torch.from_numpy(occ).cuda())
    assert np.array_equal(a, f.dense().cpu().numpy())


def test_capacity_error_reported():
    occ = workloads.dense_boxes(0)
    f = Field((64, 64, 32), 20, max_blocks=10)
    f.global_(torch.from_numpy(occ).cuda())
    assert f.error() == -3


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tunnel_full_extent(seed):
    occ = workloads.tunnels(seed)
    nz, ny, nx = occ.shape
    xyz, data = workloads.dense_to_blocks(occ)
    f = Field((nx, ny, nz), 32)
    f.global_blocks(torch.from_numpy(xyz).cuda(), torch.from_numpy(data).cuda())
    st = f.stats()
    assert st["error"] == 0 and st["obstacle_blocks"] == len(xyz)
    got = f.dense().cpu().numpy()
    ref = oracle.edt_separable(occ, 32)
    assert_same(got, ref, f"tunnel seed {seed}")
    # a sample by the plain definition too
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.integers(0, nx, 300), rng.integers(0, ny, 300),
                    rng.integers(0, nz, 300)], 1).astype(np.int32)
    assert np.array_equal(got[pts[:, 2], pts[:, 1], pts[:, 0]], oracle.edt_points(occ, 32, pts))


def test_thin_extents_beyond_65535_blocks_per_axis():
    # dense input and readbacks use one-dimensional grids: an extent with
    # more than 65535 blocks along y (or z) works
    for shape in [(1, 600000, 2), (600000, 1, 3)]:
        nz, ny, nx = shape
        rng = np.random.default_rng(nz)
        occ = (rng.random(shape) < 0.001).astype(np.uint8)
        f = gpu_field(occ, 5)
        assert_same(f.dense().cpu().numpy(), oracle.edt_separable(occ, 5), f"thin {shape}")
        assert np.array_equal(f.occupancy().cpu().numpy(), occ)
        assert f.error() == 0


def test_empty_block_list_then_updates():
    f = Field((40, 30, 20), 9)
    f.global_blocks(torch.zeros((0, 3), dtype=torch.int32, device="cuda"),
                    torch.zeros((0, 512), dtype=torch.uint8, device="cuda"))
    assert (f.dense().cpu().numpy() == 81).all() and f.error() == 0
    xyz = torch.tensor([[3, 4, 5], [39, 29, 19]], dtype=torch.int32, device="cuda")
    f.update(xyz, torch.ones(2, dtype=torch.uint8, device="cuda"))
    occ = np.zeros((20, 30, 40), np.uint8)
    occ[5, 4, 3] = occ[19, 29, 39] = 1
    assert_same(f.dense().cpu().numpy(), oracle.edt_separable(occ, 9), "after updates")
    assert f.error() == 0
