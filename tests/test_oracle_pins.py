"""Pins of the CPU EDT oracle against closed forms, an independent numpy
brute force of Eq. 1 on tiny grids, and invariants of the exact truncated
squared Euclidean distance field (VDB-EDT, section III: Eq. 1 limited to the
transform radius d_max; value D = d_max^2 beyond it; zero on obstacles)."""
import itertools

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.filterwarnings("ignore")


def closed_form(shape, obstacles, dmax):
    """min(D, min over listed obstacles of |x - o|^2) by broadcasting."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    best = np.full(shape, dmax * dmax, dtype=np.int64)
    for (ox, oy, oz) in obstacles:
        best = np.minimum(best, (x - ox) ** 2 + (y - oy) ** 2 + (z - oz) ** 2)
    return best.astype(np.int32)


def numpy_allpairs(occ, dmax):
    """Eq. 1 by an all-pairs numpy minimum (independent of the C code)."""
    nz, ny, nx = occ.shape
    D = dmax * dmax
    obs = np.argwhere(occ)                       # (z, y, x)
    if len(obs) == 0:
        return np.full(occ.shape, D, dtype=np.int32)
    cells = np.argwhere(np.ones_like(occ, dtype=bool))
    d2 = ((cells[:, None, :] - obs[None, :, :]) ** 2).sum(-1).min(1)
    return np.minimum(d2, D).reshape(occ.shape).astype(np.int32)


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build()


FIELDS = [oracle.edt_bruteforce, oracle.edt_separable]


@pytest.mark.parametrize("fn", FIELDS)
def test_empty_is_background(fn):
    occ = np.zeros((5, 6, 7), np.uint8)
    assert (fn(occ, 3) == 9).all()


@pytest.mark.parametrize("fn", FIELDS)
def test_full_is_zero(fn):
    occ = np.ones((5, 6, 7), np.uint8)
    assert (fn(occ, 3) == 0).all()


@pytest.mark.parametrize("fn", FIELDS)
@pytest.mark.parametrize("o", [(0, 0, 0), (10, 6, 4), (3, 2, 1), (10, 0, 4), (5, 6, 0)])
@pytest.mark.parametrize("dmax", [1, 2, 4, 7])
def test_single_obstacle_closed_form(fn, o, dmax):
    shape = (5, 7, 11)                            # nz, ny, nx: no two sides equal
    occ = np.zeros(shape, np.uint8)
    occ[o[2], o[1], o[0]] = 1
    assert np.array_equal(fn(occ, dmax), closed_form(shape, [o], dmax))


@pytest.mark.parametrize("fn", FIELDS)
def test_two_obstacles_closed_form(fn):
    shape = (9, 10, 13)
    obs = [(1, 2, 3), (11, 7, 5)]
    occ = np.zeros(shape, np.uint8)
    for (x, y, z) in obs:
        occ[z, y, x] = 1
    for dmax in (3, 5, 9, 20):
        assert np.array_equal(fn(occ, dmax), closed_form(shape, obs, dmax))


@pytest.mark.parametrize("fn", FIELDS)
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_closed_form(fn, axis):
    shape = (12, 13, 14)
    c = 4
    occ = np.zeros(shape, np.uint8)
    idx = [slice(None)] * 3
    idx[axis] = c
    occ[tuple(idx)] = 1
    dmax = 5
    coord = np.arange(shape[axis])
    prof = np.minimum((coord - c) ** 2, dmax * dmax)
    bshape = [1, 1, 1]
    bshape[axis] = shape[axis]
    expect = np.broadcast_to(prof.reshape(bshape), shape)
    assert np.array_equal(fn(occ, dmax), expect)


@pytest.mark.parametrize("fn", FIELDS)
def test_truncation_boundary(fn):
    # obstacle at x=0 of a 1-row grid: value (x)^2 up to D, D exactly at x=dmax
    occ = np.zeros((1, 1, 12), np.uint8)
    occ[0, 0, 0] = 1
    s = fn(occ, 5)[0, 0]
    assert list(s) == [0, 1, 4, 9, 16, 25, 25, 25, 25, 25, 25, 25]


@pytest.mark.parametrize("seed", range(40))
def test_both_match_numpy_allpairs(seed):
    rng = np.random.default_rng(1000 + seed)
    shape = tuple(int(v) for v in rng.integers(1, 13, size=3))
    p = float(rng.choice([0.0, 0.002, 0.02, 0.1, 0.4, 0.9]))
    occ = (rng.random(shape) < p).astype(np.uint8)
    dmax = int(rng.integers(1, 15))
    ref = numpy_allpairs(occ, dmax)
    assert np.array_equal(oracle.edt_bruteforce(occ, dmax), ref)
    assert np.array_equal(oracle.edt_separable(occ, dmax), ref)


@pytest.mark.parametrize("seed", range(6))
def test_separable_equals_bruteforce_medium(seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in rng.integers(8, 40, size=3))
    occ = (rng.random(shape) < rng.uniform(0.001, 0.05)).astype(np.uint8)
    for dmax in (1, 3, 8, 20):
        assert np.array_equal(oracle.edt_separable(occ, dmax),
                              oracle.edt_bruteforce(occ, dmax))


def test_points_match_field_and_out_of_extent():
    occ = workloads.dense_boxes(3, nx=24, ny=20, nz=16, p=0.01)
    dmax = 6
    full = oracle.edt_separable(occ, dmax)
    rng = np.random.default_rng(0)
    xyz = np.stack([rng.integers(-3, 27, 500), rng.integers(-3, 23, 500),
                    rng.integers(-3, 19, 500)], axis=1)
    got = oracle.edt_points(occ, dmax, xyz)
    for (x, y, z), g in zip(xyz, got):
        inside = 0 <= x < 24 and 0 <= y < 20 and 0 <= z < 16
        assert g == (full[z, y, x] if inside else 36)


def test_dense_boxes_windows_by_points():
    """Every 16^3 window of the 64x64x32 map: the definition at each voxel of
    the window (obstacles from the whole map) equals the separable field."""
    occ = workloads.dense_boxes(0)
    dmax = 20
    full = oracle.edt_separable(occ, dmax)
    for (x0, y0, z0) in itertools.product(range(0, 64, 16), range(0, 64, 16), range(0, 32, 16)):
        z, y, x = np.meshgrid(np.arange(z0, z0 + 16), np.arange(y0, y0 + 16),
                              np.arange(x0, x0 + 16), indexing="ij")
        xyz = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
        got = oracle.edt_points(occ, dmax, xyz).reshape(16, 16, 16)
        assert np.array_equal(got, full[z0:z0 + 16, y0:y0 + 16, x0:x0 + 16])


def _sum_of_three_squares(v):
    """Legendre: v >= 0 is a sum of three squares iff v != 4^a (8b + 7)."""
    v = np.asarray(v, dtype=np.int64).copy()
    nz = v > 0
    while True:
        m = nz & (v % 4 == 0)
        if not m.any():
            break
        v[m] //= 4
    return ~(nz & (v % 8 == 7))


def _lipschitz_ok(a, b, c):
    """sqrt(a) <= sqrt(b) + sqrt(c) for integers, exactly:
    a - b - c <= 0  or  (a - b - c)^2 <= 4 b c."""
    a, b = np.maximum(a, b), np.minimum(a, b)
    t = a.astype(np.int64) - b - c
    return (t <= 0) | (t * t <= 4 * b.astype(np.int64) * c)


def _invariants(occ, s, dmax):
    D = dmax * dmax
    assert s.min() >= 0 and s.max() <= D
    assert np.array_equal(s == 0, occ != 0)
    below = s[s < D]
    assert _sum_of_three_squares(below).all()
    nz, ny, nx = s.shape
    for dz, dy, dx in itertools.product((0, 1), (-1, 0, 1), (-1, 0, 1)):
        if (dz, dy, dx) <= (0, 0, 0):
            continue
        c = dz * dz + dy * dy + dx * dx
        za, zb = slice(0, nz - dz), slice(dz, nz)
        ya = slice(max(0, -dy), ny - max(0, dy)); yb = slice(max(0, dy), ny - max(0, -dy))
        xa = slice(max(0, -dx), nx - max(0, dx)); xb = slice(max(0, dx), nx - max(0, -dx))
        assert _lipschitz_ok(s[za, ya, xa], s[zb, yb, xb], c).all()


@pytest.mark.parametrize("seed", range(3))
def test_invariants_dense_boxes(seed):
    occ = workloads.dense_boxes(seed)
    _invariants(occ, oracle.edt_separable(occ, 20), 20)


@pytest.mark.parametrize("seed", range(4))
def test_invariants_sparse_random(seed):
    occ = workloads.random_grid(seed, (40, 48, 56), 0.0005)
    _invariants(occ, oracle.edt_separable(occ, 12), 12)


def test_witness_exists():
    """Each s < D is attained by some obstacle at exactly that squared
    distance, and no obstacle is closer (checked by brute force)."""
    occ = workloads.random_grid(7, (14, 15, 16), 0.01)
    dmax = 9
    s = oracle.edt_separable(occ, dmax)
    obs = np.argwhere(occ)
    cells = np.argwhere(np.ones_like(occ, dtype=bool))
    d2 = ((cells[:, None, :] - obs[None, :, :]) ** 2).sum(-1)
    flat = s.reshape(-1)
    for i in range(len(cells)):
        if flat[i] < dmax * dmax:
            assert (d2[i] == flat[i]).any() and d2[i].min() == flat[i]
        else:
            assert d2[i].min() >= dmax * dmax


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry(axis):
    occ = workloads.random_grid(11, (18, 21, 25), 0.004)
    s = oracle.edt_separable(occ, 7)
    sf = oracle.edt_separable(np.flip(occ, axis), 7)
    assert np.array_equal(np.flip(s, axis), sf)


def test_axis_permutation_on_cube():
    occ = workloads.random_grid(12, (20, 20, 20), 0.003)
    s = oracle.edt_separable(occ, 8)
    for perm in itertools.permutations(range(3)):
        sp = oracle.edt_separable(np.ascontiguousarray(occ.transpose(perm)), 8)
        assert np.array_equal(s.transpose(perm), sp)


def test_monotone_under_add_and_remove():
    occ = workloads.random_grid(13, (16, 24, 32), 0.003)
    s0 = oracle.edt_separable(occ, 10)
    more = occ.copy()
    more[3, 5, 7] = 1
    more[12, 20, 30] = 1
    s1 = oracle.edt_separable(more, 10)
    assert (s1 <= s0).all()
    fewer = occ.copy()
    fewer[np.nonzero(occ)[0][:3], np.nonzero(occ)[1][:3], np.nonzero(occ)[2][:3]] = 0
    s2 = oracle.edt_separable(fewer, 10)
    assert (s2 >= s0).all()


def test_locality_of_change():
    """Voxels farther than d_max from a changed voxel keep their value."""
    occ = workloads.random_grid(14, (24, 40, 48), 0.002)
    dmax = 6
    s0 = oracle.edt_separable(occ, dmax)
    occ2 = occ.copy()
    occ2[10, 20, 24] ^= 1
    s1 = oracle.edt_separable(occ2, dmax)
    z, y, x = np.meshgrid(np.arange(24), np.arange(40), np.arange(48), indexing="ij")
    far = (x - 24) ** 2 + (y - 20) ** 2 + (z - 10) ** 2 >= dmax * dmax
    assert np.array_equal(s0[far], s1[far])


def test_bad_arguments_raise():
    with pytest.raises(ValueError):
        oracle.edt_separable(np.zeros((2, 2, 2), np.uint8), 0)


def test_points_list_matches_grid_and_closed_form():
    rng = np.random.default_rng(21)
    occ = (rng.random((11, 13, 17)) < 0.02).astype(np.uint8)
    obs = np.argwhere(occ)[:, ::-1]                     # (x, y, z)
    z, y, x = np.meshgrid(np.arange(11), np.arange(13), np.arange(17), indexing="ij")
    xyz = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    for dmax in (1, 4, 30):
        got = oracle.edt_points_list(obs, dmax, xyz).reshape(occ.shape)
        assert np.array_equal(got, oracle.edt_bruteforce(occ, dmax))
    # one obstacle far out on a huge extent: the closed form
    o = np.array([[1_000_000, 5, 700_000]])
    q = np.array([[1_000_003, 1, 700_000], [999_990, 5, 700_012], [0, 0, 0]])
    assert list(oracle.edt_points_list(o, 20, q)) == [25, 244, 400]
    assert list(oracle.edt_points_list(np.zeros((0, 3)), 9, q)) == [81, 81, 81]


def test_uncapped_closed_forms():
    # one obstacle at the end of a long row: x^2, far beyond 16-bit values
    occ = np.zeros((3, 3, 400), np.uint8)
    occ[1, 1, 0] = 1
    u = oracle.edt_uncapped(occ)
    z, y, x = np.meshgrid(np.arange(3), np.arange(3), np.arange(400), indexing="ij")
    assert np.array_equal(u, x ** 2 + (y - 1) ** 2 + (z - 1) ** 2)
    assert u.max() == 399 ** 2 + 2
    # two obstacles: the nearer one, all-pairs
    rng = np.random.default_rng(5)
    occ = (rng.random((9, 40, 33)) < 0.002).astype(np.uint8)
    occ[0, 0, 0] = 1
    obs = np.argwhere(occ)[:, ::-1]
    zz, yy, xx = np.meshgrid(np.arange(9), np.arange(40), np.arange(33), indexing="ij")
    q = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
    want = oracle.edt_points_list(obs, 46340, q).reshape(occ.shape)
    assert np.array_equal(oracle.edt_uncapped(occ), want)
    assert (oracle.edt_uncapped(np.zeros((4, 5, 6), np.uint8)) == oracle.INF).all()
