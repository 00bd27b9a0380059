"""Pins of the oracle's scan integration: the integer voxel walk against
exact geometry (every voxel whose open cube the segment crosses is visited,
every visited voxel's closed cube touches the segment), its shape (length,
ends, 6-connected, monotone), the tie order on diagonals, and the free / hit
marking of a scan on small grids."""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def seg_hits_cube(o, e, v, open_cube):
    """Exact test: does the segment between voxel centres o and e meet the
    cube of voxel v (open or closed)?  Liang-Barsky with fractions."""
    t0, t1 = Fraction(0), Fraction(1)
    for a in range(3):
        d = e[a] - o[a]
        lo, hi = Fraction(2 * v[a] - 1, 2), Fraction(2 * v[a] + 1, 2)
        if d == 0:
            if open_cube and not (lo < o[a] < hi):
                return False
            if not open_cube and not (lo <= o[a] <= hi):
                return False
            continue
        ta, tb = (lo - o[a]) / d, (hi - o[a]) / d
        if ta > tb:
            ta, tb = tb, ta
        t0, t1 = max(t0, ta), min(t1, tb)
    return t0 < t1 if open_cube else t0 <= t1


@pytest.mark.parametrize("seed", range(6))
def test_walk_against_geometry(seed):
    rng = np.random.default_rng(seed)
    for _ in range(40):
        o = rng.integers(0, 9, 3)
        e = o + rng.integers(-7, 8, 3)
        path = oracle.ray_voxels(o, e)
        vis = {tuple(v) for v in path}
        lo, hi = np.minimum(o, e), np.maximum(o, e)
        for v in np.ndindex(*(hi - lo + 1)):
            v = tuple(int(c) for c in np.array(v) + lo)
            if seg_hits_cube(o, e, v, open_cube=True):
                assert v in vis, (o, e, v)
        for v in vis:
            assert seg_hits_cube(o, e, v, open_cube=False), (o, e, v)


def test_walk_shape():
    rng = np.random.default_rng(11)
    for _ in range(300):
        o = rng.integers(-50, 50, 3)
        e = o + rng.integers(-60, 61, 3)
        p = oracle.ray_voxels(o, e).astype(np.int64)
        assert len(p) == np.abs(e - o).sum() + 1
        assert (p[0] == o).all() and (p[-1] == e).all()
        step = np.diff(p, axis=0)
        assert (np.abs(step).sum(1) == 1).all()          # 6-connected, one axis per step
        sgn = np.sign(e - o)
        assert ((step * sgn) >= 0).all()                  # monotone toward e


def test_axis_rays_and_tie_order():
    p = oracle.ray_voxels([2, 3, 4], [2, 3, 9])
    assert p.tolist() == [[2, 3, z] for z in range(4, 10)]
    p = oracle.ray_voxels([5, 0, 0], [1, 0, 0])
    assert p.tolist() == [[x, 0, 0] for x in range(5, 0, -1)]
    # equal crossing parameters: x, then y, then z
    assert oracle.ray_voxels([0, 0, 0], [2, 2, 2]).tolist() == [
        [0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1], [2, 1, 1], [2, 2, 1], [2, 2, 2]]
    assert oracle.ray_voxels([0, 0, 0], [-1, 0, 1]).tolist() == [[0, 0, 0], [-1, 0, 0], [-1, 0, 1]]
    # crossings at 1/4 and 3/4 on x against 1/2 on y
    assert oracle.ray_voxels([0, 0, 0], [2, 1, 0]).tolist() == [[0, 0, 0], [1, 0, 0], [1, 1, 0],
                                                                 [2, 1, 0]]


def test_integrate_marking():
    occ = np.zeros((4, 5, 9), np.uint8)       # (nz, ny, nx)
    occ[0, 0, 4] = 1                          # on ray 0's path: cleared
    occ[0, 2, 8] = 1                          # end of ray 1 without a return: cleared
    origin = [0, 0, 0]
    ends = np.array([[6, 0, 0], [8, 2, 0], [3, 0, 0], [9, 0, 0], [2, 4, 3]])
    hits = np.array([1, 0, 1, 1, 0], np.uint8)
    new, skipped = oracle.integrate_scan(occ, origin, ends, hits)
    assert skipped == 1                       # (9, 0, 0) is outside
    assert new[0, 0, 6] == 1                  # hit of ray 0
    assert new[0, 0, 3] == 1                  # hit of ray 2 wins over ray 0 passing through
    assert new[0, 0, 4] == 0 and new[0, 2, 8] == 0
    # the same marking from the walks, by hand
    want = occ.copy()
    free, hit = set(), set()
    for e, h in zip(ends, hits):
        if (e < 0).any() or (e >= [9, 5, 4]).any():
            continue
        free |= {tuple(v) for v in oracle.ray_voxels(origin, e)}
        if h:
            hit.add(tuple(e))
    for x, y, z in free:
        want[z, y, x] = 0
    for x, y, z in hit:
        want[z, y, x] = 1
    assert np.array_equal(new, want)


def test_integrate_origin_outside_skips_everything():
    occ = np.ones((3, 3, 3), np.uint8)
    new, skipped = oracle.integrate_scan(occ, [-1, 0, 0], np.array([[1, 1, 1], [2, 2, 2]]),
                                         np.array([0, 1], np.uint8))
    assert skipped == 2 and np.array_equal(new, occ)
