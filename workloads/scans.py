"""Simulated range scans that drive the incremental transform.

A world W_t and a map M_t start equal to the initial occupancy.  Scan t:
  1. pose: the point at arc length `advance * t` along the given path
     (polyline points one voxel apart, wrapping), rounded to a voxel;
  2. dynamics: in W, toggle `toggle_frac` of the original wall voxels that
     lie within `max_range` of the pose (seeded by (seed, t));
  3. rays: `n_elev` elevations evenly spaced in [-elev_deg, +elev_deg] times
     `n_azim` azimuths k * 360 / n_azim, traversed voxel by voxel
     (Amanatides & Woo) from the pose voxel's center; a ray stops at the
     first voxel occupied in W_t (a hit), once the path length at which it
     enters a voxel exceeds `max_range`, or at the extent boundary;
  4. map: traversed voxels become free in M, hits become occupied (a hit in
     any ray wins over a traversal by another);
  5. the change list is {v : M_{t+1}(v) != M_t(v)} with the new states.
This is harness code (it stands in for the LIDAR datasets of the paper's
section V-B); it holds no distance-transform arithmetic.
"""
from __future__ import annotations

import numpy as np


def ray_directions(n_elev=16, n_azim=1024, elev_deg=15.0):
    el = np.deg2rad(np.linspace(-elev_deg, elev_deg, n_elev))
    az = 2 * np.pi * np.arange(n_azim) / n_azim
    E, A = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)
    return d.reshape(-1, 3)


def cast_rays(world: np.ndarray, origin, dirs: np.ndarray, max_range: float,
              ends: bool = False):
    """Voxel traversal of all rays at once.  Returns (traversed linear indices,
    hit linear indices), both possibly with repeats; with ends=True also each
    ray's last voxel (x, y, z), int32[n, 3], and whether it ended on a hit."""
    nz, ny, nx = world.shape
    flat = world.reshape(-1)
    n = len(dirs)
    o = np.asarray(origin, dtype=np.float64)
    vox = np.tile(np.round(o).astype(np.int64), (n, 1))
    step = np.where(dirs >= 0, 1, -1).astype(np.int64)
    with np.errstate(divide="ignore"):
        inv = np.where(dirs != 0, 1.0 / np.abs(dirs), np.inf)
    # distance along the ray to the first voxel face on each axis
    tmax = np.where(dirs != 0, (vox + 0.5 * step - o) * step * inv, np.inf)
    alive = np.ones(n, dtype=bool)
    ext = np.array([nx, ny, nz])
    trav, hits = [], []
    idx = np.arange(n)
    last = vox.copy()
    hit_ray = np.zeros(n, dtype=bool)
    while alive.any():
        a = idx[alive]
        v = vox[a]
        inside = ((v >= 0) & (v < ext)).all(1)
        alive[a[~inside]] = False
        a, v = a[inside], v[inside]
        if len(a) == 0:
            break
        lin = v[:, 0] + nx * (v[:, 1] + ny * v[:, 2])
        last[a] = v
        occ = flat[lin] != 0
        hits.append(lin[occ])
        hit_ray[a[occ]] = True
        alive[a[occ]] = False
        a, lin = a[~occ], lin[~occ]
        trav.append(lin)
        tm = tmax[a]
        ax = np.argmin(tm, axis=1)
        t_enter = tm[np.arange(len(a)), ax]
        vox[a, ax] += step[a, ax]
        tmax[a, ax] += inv[a, ax]
        alive[a[t_enter > max_range]] = False
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0, np.int64)
    if ends:
        return cat(trav), cat(hits), last.astype(np.int32), hit_ray.astype(np.uint8)
    return cat(trav), cat(hits)


class ScanSim:
    def __init__(self, occ0: np.ndarray, path: np.ndarray, seed: int, advance=40.0,
                 max_range=150.0, n_elev=16, n_azim=1024, elev_deg=15.0,
                 toggle_frac=0.02, toggle_scope="local"):
        self.world = occ0.copy()
        self.map = occ0.copy()
        self.walls = np.flatnonzero(occ0.reshape(-1))
        nz, ny, nx = occ0.shape
        self.shape = occ0.shape
        wz = self.walls // (nx * ny)
        wy = (self.walls // nx) % ny
        wx = self.walls % nx
        self.wall_xyz = np.stack([wx, wy, wz], 1)
        self.path = np.asarray(path, dtype=np.float64)
        self.seed = seed
        self.advance = advance
        self.max_range = max_range
        self.dirs = ray_directions(n_elev, n_azim, elev_deg)
        self.toggle_frac = toggle_frac
        self.toggle_scope = toggle_scope
        self.t = 0

    def pose(self, t):
        k = int(round(self.advance * t)) % len(self.path)
        nz, ny, nx = self.shape
        p = np.round(self.path[k]).astype(np.int64)
        return np.clip(p, 0, [nx - 1, ny - 1, nz - 1])

    def rays(self):
        """Advance one scan of the world only and return the rays as a sensor
        reports them: (pose int32[3], end voxels int32[n, 3], hits uint8[n]).
        The map is left to the caller (occupancy integration)."""
        t = self.t
        self.t += 1
        rng = np.random.default_rng([self.seed, t])
        pose = self.pose(t)
        self._toggle(rng, pose)
        _, _, last, hit = cast_rays(self.world, pose, self.dirs, self.max_range, ends=True)
        return pose.astype(np.int32), last, hit

    def _toggle(self, rng, pose):
        if self.toggle_scope == "global":
            cand = self.walls
        else:
            d2 = ((self.wall_xyz - pose) ** 2).sum(1)
            cand = self.walls[d2 <= self.max_range ** 2]
        k = int(round(self.toggle_frac * len(cand)))
        if k:
            flip = rng.choice(cand, size=k, replace=False)
            w = self.world.reshape(-1)
            w[flip] ^= 1

    def step(self):
        """Advance one scan.  Returns (xyz int32[n, 3], state uint8[n], pose)."""
        t = self.t
        self.t += 1
        rng = np.random.default_rng([self.seed, t])
        pose = self.pose(t)
        self._toggle(rng, pose)
        trav, hits = cast_rays(self.world, pose, self.dirs, self.max_range)
        touched = np.unique(np.concatenate([trav, hits]))
        m = self.map.reshape(-1)
        old = m[touched].copy()
        m[trav] = 0
        m[hits] = 1
        new = m[touched]
        ch = touched[new != old]
        nz, ny, nx = self.shape
        xyz = np.stack([ch % nx, (ch // nx) % ny, ch // (nx * ny)], 1).astype(np.int32)
        return xyz, m[ch].astype(np.uint8), pose


def tunnel_path(seed: int, **kw) -> np.ndarray:
    """Centerlines of the tunnel map concatenated in index order."""
    from . import tunnel_centerlines
    return np.concatenate([pts for pts, _ in tunnel_centerlines(seed, **kw)])


def ellipse_path(nx, ny, nz, n=2048):
    """Closed loop in the plane z = nz/2 used for scans of small dense maps."""
    a = 2 * np.pi * np.arange(n) / n
    cx, cy = (nx - 1) / 2, (ny - 1) / 2
    rx, ry = 0.3 * nx, 0.3 * ny
    pts = np.stack([cx + rx * np.cos(a), cy + ry * np.sin(a), np.full(n, nz / 2)], 1)
    # resample to ~1 voxel spacing
    seg = np.linalg.norm(np.diff(pts, axis=0), axis=1)
    s = np.concatenate([[0], np.cumsum(seg)])
    u = np.arange(0, s[-1], 1.0)
    return np.stack([np.interp(u, s, pts[:, i]) for i in range(3)], 1)
