"""Pins of the oracle's interior distances and signed field (the definition
with occupied and free voxels exchanged): closed forms for boxes and slabs,
numpy all-pairs brute force on small random grids, the empty and full
extents, and the reading that voxels outside the extent are not free."""
import numpy as np
import pytest

import oracle


def allpairs_interior(occ, dmax):
    """Brute force: for every voxel, the least squared distance to a free
    voxel of the grid, clamped to D (D where there is none)."""
    free = np.argwhere(occ == 0)
    pts = np.argwhere(np.ones_like(occ))
    out = np.full(occ.shape, dmax * dmax, dtype=np.int64)
    if len(free):
        d2 = ((pts[:, None, :] - free[None, :, :]) ** 2).sum(-1).min(1)
        out = np.minimum(d2, dmax * dmax).reshape(occ.shape)
    return out


@pytest.mark.parametrize("seed,p,dmax", [(0, 0.5, 3), (1, 0.8, 5), (2, 0.95, 9), (3, 0.3, 2),
                                         (4, 0.99, 12), (5, 0.7, 1)])
def test_interior_matches_allpairs(seed, p, dmax):
    rng = np.random.default_rng(seed)
    occ = (rng.random((7, 9, 11)) < p).astype(np.uint8)
    ref = allpairs_interior(occ, dmax)
    assert np.array_equal(oracle.interior(occ, dmax)[occ != 0], ref[occ != 0])


def test_box_closed_form():
    nz, ny, nx = 18, 22, 26
    lo, hi = np.array([3, 4, 5]), np.array([12, 15, 17])      # (z, y, x), inclusive
    occ = np.zeros((nz, ny, nx), np.uint8)
    occ[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] = 1
    for dmax in (2, 4, 30):
        D = dmax * dmax
        sf = oracle.signed_field(occ, dmax)
        for z, y, x in np.ndindex(nz, ny, nx):
            v = np.array([z, y, x])
            if occ[z, y, x]:
                # nearest free voxel: just outside the nearest face, one axis
                d = min(min(v[a] - lo[a] + 1, hi[a] + 1 - v[a]) for a in range(3))
                want = -min(D, d * d)
            else:
                gap = np.maximum(np.maximum(lo - v, 0), np.maximum(v - hi, 0))
                want = min(D, int((gap ** 2).sum()))
            assert sf[z, y, x] == want, (z, y, x, dmax)


def test_outside_the_extent_is_not_free():
    # a slab across the whole x and y extent: free voxels only above and below
    occ = np.zeros((16, 6, 5), np.uint8)
    occ[4:12] = 1
    sf = oracle.signed_field(occ, 10)
    for z in range(4, 12):
        d = min(z - 3, 12 - z)
        assert (sf[z] == -d * d).all()
    # the whole extent occupied: no free voxel at all
    full = np.ones((4, 5, 6), np.uint8)
    assert (oracle.signed_field(full, 7) == -49).all()


def test_empty_extent_and_single_free_voxel():
    assert (oracle.signed_field(np.zeros((3, 4, 5), np.uint8), 6) == 36).all()
    occ = np.ones((9, 9, 9), np.uint8)
    occ[2, 5, 7] = 0
    sf = oracle.signed_field(occ, 6)
    z, y, x = np.meshgrid(np.arange(9), np.arange(9), np.arange(9), indexing="ij")
    want = -np.minimum((z - 2) ** 2 + (y - 5) ** 2 + (x - 7) ** 2, 36)
    want[2, 5, 7] = 1      # the free voxel itself: its six face neighbours are obstacles
    assert np.array_equal(sf, want)


def test_sign_and_range():
    rng = np.random.default_rng(9)
    occ = (rng.random((12, 13, 14)) < 0.5).astype(np.uint8)
    sf = oracle.signed_field(occ, 8)
    assert (sf[occ != 0] <= -1).all() and (sf[occ != 0] >= -64).all()
    assert (sf[occ == 0] >= 1).all() and (sf[occ == 0] <= 64).all()
    # a boundary voxel (occupied with a free 6-neighbour) is at -1, and only those
    pad = np.pad(occ, 1, constant_values=1)
    free_nb = np.zeros_like(occ, bool)
    for a in range(3):
        for s in (-1, 1):
            free_nb |= np.roll(pad == 0, s, axis=a)[1:-1, 1:-1, 1:-1]
    assert np.array_equal(sf[occ != 0] == -1, free_nb[occ != 0])
