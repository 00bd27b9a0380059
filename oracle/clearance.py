"""Clearance cost oracle in float64 -- test infrastructure only.

The paper's planning objective (section III, Eq. 2) penalises waypoints that
come closer than a margin to obstacles through the distance field d(x).  The
form computed here is the squared hinge

    c(p) = max(0, m - d(p))^2,      C_t = sum over waypoints p of trajectory t,

with d(p) the trilinear interpolation of the metric distance field
d_m(i) = h * sqrt(s(i)) (s = truncated squared voxel distance, h = voxel
edge in metres).  Voxel center i sits at metric position i * h.

Per axis with grid size n and u = p / h:
    i0 = clamp(floor(u), 0, n - 2),   t = clamp(u - i0, 0, 1);
an axis whose t was clamped contributes no gradient (the interpolant is
constant there).  Everything is float64; fp32 inputs are widened exactly.
"""
from __future__ import annotations

import numpy as np


def metric_field(s: np.ndarray, h: float) -> np.ndarray:
    """d_m = h * sqrt(s) in float64, s is the int32 squared-distance field."""
    return float(h) * np.sqrt(np.asarray(s, dtype=np.float64))


def _axis(u: np.ndarray, n: int):
    """Cell index, cell coordinate and 'not clamped' flag along one axis."""
    i0 = np.clip(np.floor(u), 0, n - 2).astype(np.int64)
    t_raw = u - i0
    t = np.clip(t_raw, 0.0, 1.0)
    live = (t_raw >= 0.0) & (t_raw <= 1.0)
    return i0, t, live


def trilinear(field: np.ndarray, p: np.ndarray, h: float):
    """Value and gradient (d/dp, metres) of the trilinear interpolant of a
    (nz, ny, nx) float64 field at points p[..., 3] = (x, y, z) metres."""
    field = np.asarray(field, dtype=np.float64)
    nz, ny, nx = field.shape
    p = np.asarray(p, dtype=np.float64)
    u = p / float(h)
    ix, tx, lx = _axis(u[..., 0], nx)
    iy, ty, ly = _axis(u[..., 1], ny)
    iz, tz, lz = _axis(u[..., 2], nz)

    def f(dz, dy, dx):
        return field[iz + dz, iy + dy, ix + dx]

    c000, c001, c010, c011 = f(0, 0, 0), f(0, 0, 1), f(0, 1, 0), f(0, 1, 1)
    c100, c101, c110, c111 = f(1, 0, 0), f(1, 0, 1), f(1, 1, 0), f(1, 1, 1)
    wx0, wy0, wz0 = 1.0 - tx, 1.0 - ty, 1.0 - tz
    val = (wz0 * (wy0 * (wx0 * c000 + tx * c001) + ty * (wx0 * c010 + tx * c011)) +
           tz * (wy0 * (wx0 * c100 + tx * c101) + ty * (wx0 * c110 + tx * c111)))
    gx = (wz0 * (wy0 * (c001 - c000) + ty * (c011 - c010)) +
          tz * (wy0 * (c101 - c100) + ty * (c111 - c110)))
    gy = (wz0 * (wx0 * (c010 - c000) + tx * (c011 - c001)) +
          tz * (wx0 * (c110 - c100) + tx * (c111 - c101)))
    gz = (wy0 * (wx0 * (c100 - c000) + tx * (c101 - c001)) +
          ty * (wx0 * (c110 - c010) + tx * (c111 - c011)))
    grad = np.stack([gx * lx, gy * ly, gz * lz], axis=-1) / float(h)
    return val, grad


def cost(s: np.ndarray, wp: np.ndarray, h: float, margin: float):
    """Per-trajectory cost C_t (float64 [T]) for waypoints wp[T, W, 3]."""
    d, _ = trilinear(metric_field(s, h), wp, h)
    c = np.maximum(0.0, margin - d) ** 2
    return c.sum(axis=-1)


def cost_grad(s: np.ndarray, wp: np.ndarray, h: float, margin: float,
              gcost: np.ndarray | None = None):
    """Analytic dL/dwp for L = sum_t gcost[t] * C_t (gcost defaults to ones)."""
    d, gd = trilinear(metric_field(s, h), wp, h)
    hinge = np.maximum(0.0, margin - d)
    g = -2.0 * hinge[..., None] * gd
    if gcost is not None:
        g = g * np.asarray(gcost, dtype=np.float64)[:, None, None]
    return g


def cost_grad_fd(s: np.ndarray, wp: np.ndarray, h: float, margin: float,
                 eps: float = 1e-4):
    """Central finite differences of C_t with respect to every coordinate."""
    field = metric_field(s, h)
    wp = np.asarray(wp, dtype=np.float64)

    def c_pt(p):
        d, _ = trilinear(field, p, h)
        return np.maximum(0.0, margin - d) ** 2

    g = np.empty_like(wp)
    for a in range(3):
        e = np.zeros(3)
        e[a] = eps
        g[..., a] = (c_pt(wp + e) - c_pt(wp - e)) / (2.0 * eps)
    return g
