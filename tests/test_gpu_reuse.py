"""One field reused for a second map.  The passes do not store g1 or g2 for
blocks that are D everywhere (their readers take the shared D block), so
after a map whose blocks were all stored, the pool still holds that map's
values where the next map's skipped blocks now live.  The transform, the
nearest-obstacle query and incremental updates must never read them."""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_04419_amd import Field
from test_gpu_nearest import all_voxels, check_nearest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available()
    oracle.build(force=False)


def sparse_map(rng, nx, ny, nz):
    """A few small boxes and isolated voxels: most region blocks are D
    everywhere after pass X, and whole columns after pass Y."""
    occ = np.zeros((nz, ny, nx), np.uint8)
    for _ in range(3):
        x, y, z = rng.integers(0, nx - 4), rng.integers(0, ny - 4), rng.integers(0, nz - 4)
        occ[z:z + 3, y:y + 2, x:x + 4] = 1
    for _ in range(4):
        occ[rng.integers(0, nz), rng.integers(0, ny), rng.integers(0, nx)] = 1
    return occ


@pytest.mark.parametrize("dmax", [16, 32, 100])
def test_sparse_map_after_dense_map(dmax):
    rng = np.random.default_rng(dmax)
    nx, ny, nz = 96, 80, 48
    D = dmax * dmax
    f = Field((nx, ny, nz), dmax)
    dense_occ = (rng.random((nz, ny, nx)) < 0.2).astype(np.uint8)
    f.global_(torch.from_numpy(dense_occ).cuda())
    assert np.array_equal(f.dense().cpu().numpy(), oracle.edt_separable(dense_occ, dmax))

    occ = sparse_map(rng, nx, ny, nz)
    f.global_(torch.from_numpy(occ).cuda())
    ref = oracle.edt_separable(occ, dmax)
    assert np.array_equal(f.dense().cpu().numpy(), ref), "global transform after a dense map"
    xyz = all_voxels(nx, ny, nz)
    got = f.query_nearest(torch.from_numpy(xyz).cuda()).cpu().numpy()
    check_nearest(occ, ref.reshape(-1), xyz, got, D, f"nearest after a dense map d={dmax}")

    # updates that put obstacles where blocks were D everywhere and take
    # some away: the update recomputes blocks next to skipped ones
    for step in range(4):
        n = 40
        cx = rng.integers(0, nx, n).astype(np.int32)
        cy = rng.integers(0, ny, n).astype(np.int32)
        cz = rng.integers(0, nz, n).astype(np.int32)
        st = (rng.random(n) < 0.7).astype(np.uint8)
        occ[cz, cy, cx] = 0
        for i in range(n):
            occ[cz[i], cy[i], cx[i]] = st[i]
        f.update(torch.from_numpy(np.stack([cx, cy, cz], 1)).cuda(), torch.from_numpy(st).cuda())
        ref = oracle.edt_separable(occ, dmax)
        assert np.array_equal(f.dense().cpu().numpy(), ref), f"update {step} d={dmax}"
    got = f.query_nearest(torch.from_numpy(xyz).cuda()).cpu().numpy()
    check_nearest(occ, ref.reshape(-1), xyz, got, D, f"nearest after updates d={dmax}")
