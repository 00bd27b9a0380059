"""Pins of the float64 clearance oracle (VDB-EDT section III, Eq. 2 clearance
term in squared-hinge form, on a trilinear interpolant of the field)."""
import numpy as np
import pytest

from oracle import clearance as cl

H = 0.2


def test_metric_field_perfect_squares():
    s = np.array([0, 1, 4, 9, 400], dtype=np.int32).reshape(1, 1, 5)
    assert np.array_equal(cl.metric_field(s, H), H * np.array([0, 1, 2, 3, 20.0]).reshape(1, 1, 5))


def test_interpolates_voxel_centers():
    rng = np.random.default_rng(0)
    f = rng.random((5, 6, 7))
    z, y, x = np.meshgrid(np.arange(5), np.arange(6), np.arange(7), indexing="ij")
    p = np.stack([x, y, z], -1).astype(np.float64) * H
    v, _ = cl.trilinear(f, p, H)
    assert np.allclose(v, f, rtol=0, atol=1e-12)


def test_linear_field_is_reproduced():
    """Trilinear interpolation reproduces an affine field exactly, with the
    affine gradient divided by h; distinct slopes per axis on a non-cubic
    grid catch any axis transposition."""
    nz, ny, nx = 6, 8, 10
    a, b, c, e = 0.7, -1.3, 2.9, 5.0
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = a * x + b * y + c * z + e
    rng = np.random.default_rng(1)
    u = rng.random((200, 3)) * np.array([nx - 1, ny - 1, nz - 1])
    v, g = cl.trilinear(f, u * H, H)
    assert np.allclose(v, a * u[:, 0] + b * u[:, 1] + c * u[:, 2] + e, atol=1e-12)
    assert np.allclose(g, np.array([a, b, c]) / H, atol=1e-9)


def test_clamped_axis_has_zero_gradient():
    f = np.random.default_rng(2).random((4, 5, 6))
    p = np.array([[-0.3, 0.31, 0.27], [0.5, 9.0, 0.2], [0.41, 0.33, 5.0]])
    _, g = cl.trilinear(f, p, H)
    assert g[0, 0] == 0 and g[1, 1] == 0 and g[2, 2] == 0
    assert g[0, 1] != 0 and g[1, 0] != 0 and g[2, 0] != 0


def test_constant_field_no_gradient_and_far_is_free():
    s = np.full((6, 6, 6), 400, dtype=np.int32)      # d = 4 m > margin 1
    wp = np.random.default_rng(3).random((3, 5, 3)) * 1.0
    assert np.all(cl.cost(s, wp, H, 1.0) == 0)
    assert np.all(cl.cost_grad(s, wp, H, 1.0) == 0)
    s2 = np.full((6, 6, 6), 4, dtype=np.int32)       # d = 0.4 m < margin
    assert np.allclose(cl.cost(s2, wp, H, 1.0), 5 * 0.6 ** 2)
    assert np.all(cl.cost_grad(s2, wp, H, 1.0) == 0)


def test_cost_is_sum_of_hinge():
    rng = np.random.default_rng(4)
    s = rng.integers(0, 30, size=(6, 7, 8)).astype(np.int32)
    wp = rng.random((4, 9, 3)) * np.array([7, 6, 5]) * H
    f = cl.metric_field(s, H)
    tot = np.zeros(4)
    for t in range(4):
        for w in range(9):
            d, _ = cl.trilinear(f, wp[t, w][None], H)
            tot[t] += max(0.0, 1.0 - d[0]) ** 2
    assert np.allclose(cl.cost(s, wp, H, 1.0), tot, rtol=1e-14)


def test_analytic_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    s = rng.integers(0, 40, size=(10, 11, 12)).astype(np.int32)
    u = 0.5 + rng.random((64, 32, 3)) * (np.array([12, 11, 10]) - 2.0)
    wp = u * H
    eps = 1e-4
    g = cl.cost_grad(s, wp, H, 1.0)
    gfd = cl.cost_grad_fd(s, wp, H, 1.0, eps)
    d, gd = cl.trilinear(cl.metric_field(s, H), wp, H)
    frac = u - np.floor(u)
    near_face = (np.minimum(frac, 1 - frac) < 10 * eps / H).any(-1)
    near_hinge = np.abs(1.0 - d) < 10 * eps * np.linalg.norm(gd, axis=-1)
    ok = ~(near_face | near_hinge)
    assert ok.mean() > 0.9
    scale = max(np.abs(g[ok]).max(), 1e-12)
    err = np.abs(g[ok] - gfd[ok])
    assert (err <= 1e-6 * np.maximum(np.abs(g[ok]), 1e-3 * scale)).all()


def test_upstream_gradient_scales():
    rng = np.random.default_rng(6)
    s = rng.integers(0, 40, size=(6, 6, 6)).astype(np.int32)
    wp = (0.5 + rng.random((3, 4, 3)) * 4) * H
    gc = np.array([2.0, -1.0, 0.5])
    assert np.allclose(cl.cost_grad(s, wp, H, 1.0, gc),
                       cl.cost_grad(s, wp, H, 1.0) * gc[:, None, None])

