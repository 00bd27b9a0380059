"""Seeded synthetic workloads shaped like the VDB-EDT paper's maps.

This module only draws inputs: occupancy grids, sparse block lists, sensor
change lists and trajectories.  It holds none of the distance-transform
arithmetic, so both the CPU oracle and the HIP library can be fed from it
without sharing any code with each other.

Array convention: a dense map is a numpy uint8 array of shape (nz, ny, nx)
in C order, so x is the fastest axis and the linear index of voxel (x, y, z)
is x + nx * (y + ny * z).  Nonzero means occupied.

Workloads (d_max in voxels, truncation value D = d_max**2):
  dense_boxes      dense 64x64x32 grid, Bernoulli(0.05) plus 4 solid boxes
                   (paper section V-A uses random obstacles in cubic maps).
  tunnels          1024x1024x128 sparse extent, 1-voxel tube walls around 12
                   persistent random-walk centerlines (stands in for the SubT
                   tunnel dataset of section V-B, which is not available).
  batch_maps       64 dense maps, sides U{32..256}, i.i.d. density U(1%,30%)
                   unioned with recursive room layouts with door gaps.
  trajectories     clamped cubic B-splines through free voxels of a map.
  scans            simulated 360 x 30 degree range scans along a centerline
                   (module workloads.scans).
"""
from __future__ import annotations

import os
import numpy as np

__all__ = [
    "dense_boxes", "tunnels", "tunnel_centerlines", "dense_to_blocks",
    "blocks_to_dense", "batch_maps", "room_layout", "trajectories",
    "random_grid", "cache_dir",
]


def cache_dir() -> str:
    d = os.environ.get("VDBEDT_CACHE", os.path.join("/tmp", "vdbedt_cache"))
    os.makedirs(d, exist_ok=True)
    return d


# ---------------------------------------------------------------------------
# dense 64x64x32: Bernoulli field, then 4 solid boxes
# ---------------------------------------------------------------------------
def dense_boxes(seed: int, nx: int = 64, ny: int = 64, nz: int = 32,
                p: float = 0.05, nboxes: int = 4, side_lo: int = 4,
                side_hi: int = 16) -> np.ndarray:
    """Bernoulli(p) occupancy drawn first (array order), then `nboxes` solid
    axis-aligned boxes, each side uniform in {side_lo..side_hi}, the min
    corner uniform so that the box lies fully inside the grid."""
    rng = np.random.default_rng(seed)
    occ = (rng.random((nz, ny, nx)) < p).astype(np.uint8)
    for _ in range(nboxes):
        sx, sy, sz = (int(rng.integers(side_lo, side_hi + 1)) for _ in range(3))
        sx, sy, sz = min(sx, nx), min(sy, ny), min(sz, nz)
        x0 = int(rng.integers(0, nx - sx + 1))
        y0 = int(rng.integers(0, ny - sy + 1))
        z0 = int(rng.integers(0, nz - sz + 1))
        occ[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx] = 1
    return occ


def random_grid(seed: int, shape, p: float) -> np.ndarray:
    """i.i.d. Bernoulli(p) occupancy of the given (nz, ny, nx) shape."""
    rng = np.random.default_rng(seed)
    return (rng.random(shape) < p).astype(np.uint8)


# ---------------------------------------------------------------------------
# sparse tunnel map
# ---------------------------------------------------------------------------
TUNNEL_STEPS = 600   # walk length per centerline; gives ~5% allocated blocks


def tunnel_centerlines(seed: int, nx=1024, ny=1024, nz=128, ntubes=12,
                       rmin=8.0, rmax=20.0, steps=TUNNEL_STEPS):
    """Persistent random walks with unit steps.  Returns a list of
    (points float64[m+1, 3] as (x, y, z), radius).  The walk stays inside the
    extent with a margin of radius + 2 by reflecting position and heading;
    the vertical heading component is damped so tubes run mostly level."""
    rng = np.random.default_rng(seed)
    ext = np.array([nx, ny, nz], dtype=np.float64)
    tubes = []
    for _ in range(ntubes):
        r = float(rng.uniform(rmin, rmax))
        lo = np.full(3, r + 2.0)
        hi = ext - r - 3.0
        p = lo + rng.random(3) * (hi - lo)
        d = rng.normal(size=3)
        d[2] *= 0.2
        d /= np.linalg.norm(d)
        pts = [p.copy()]
        for _ in range(steps):
            d = d + 0.12 * rng.normal(size=3)
            d[2] *= 0.5
            d /= np.linalg.norm(d)
            p = p + d
            for a in range(3):
                if p[a] < lo[a]:
                    p[a] = 2 * lo[a] - p[a]
                    d[a] = -d[a]
                elif p[a] > hi[a]:
                    p[a] = 2 * hi[a] - p[a]
                    d[a] = -d[a]
            pts.append(p.copy())
        tubes.append((np.array(pts), r))
    return tubes


def _tube_walls(occ: np.ndarray, pts: np.ndarray, r: float) -> None:
    """Mark voxels v with (r-0.5)^2 <= dist(v, centerline points)^2 < (r+0.5)^2,
    distance measured from the voxel center (integer coordinates)."""
    nz, ny, nx = occ.shape
    h = int(np.ceil(r + 1.5))
    lo = np.maximum(np.floor(pts.min(0)).astype(int) - h, 0)
    hi = np.minimum(np.ceil(pts.max(0)).astype(int) + h + 1, [nx, ny, nz])
    box = np.full((hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0]), np.inf,
                  dtype=np.float32)
    for p in pts:
        c0 = np.maximum(np.floor(p).astype(int) - h, lo)
        c1 = np.minimum(np.floor(p).astype(int) + h + 1, hi)
        xs = (np.arange(c0[0], c1[0]) - p[0]) ** 2
        ys = (np.arange(c0[1], c1[1]) - p[1]) ** 2
        zs = (np.arange(c0[2], c1[2]) - p[2]) ** 2
        d2 = (zs[:, None, None] + ys[None, :, None] + xs[None, None, :]).astype(np.float32)
        sl = box[c0[2] - lo[2]:c1[2] - lo[2], c0[1] - lo[1]:c1[1] - lo[1],
                 c0[0] - lo[0]:c1[0] - lo[0]]
        np.minimum(sl, d2, out=sl)
    wall = (box >= (r - 0.5) ** 2) & (box < (r + 0.5) ** 2)
    occ[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] |= wall.astype(np.uint8)


def tunnels(seed: int, nx=1024, ny=1024, nz=128, ntubes=12, rmin=8.0,
            rmax=20.0, steps=TUNNEL_STEPS, use_cache=True) -> np.ndarray:
    """Dense uint8 occupancy (nz, ny, nx) of the tunnel map.  Cached as .npy."""
    path = os.path.join(cache_dir(), f"tunnels_s{seed}_{nx}x{ny}x{nz}_t{ntubes}_"
                        f"r{rmin:g}-{rmax:g}_w{steps}.npy")
    if use_cache and os.path.exists(path):
        return np.load(path)
    occ = np.zeros((nz, ny, nx), dtype=np.uint8)
    for pts, r in tunnel_centerlines(seed, nx, ny, nz, ntubes, rmin, rmax, steps):
        _tube_walls(occ, pts, r)
    if use_cache:
        tmp = path + f".{os.getpid()}.tmp.npy"
        np.save(tmp, occ)
        os.replace(tmp, path)
    return occ


def dense_to_blocks(occ: np.ndarray):
    """Split a dense (nz, ny, nx) map (sides multiples of 8) into 8^3 leaf
    blocks.  Returns (block_xyz int32[n, 3] as (bx, by, bz),
    block_occ uint8[n, 512] with in-block index x + 8*y + 64*z) for blocks
    holding at least one occupied voxel, in (bz, by, bx) order."""
    nz, ny, nx = occ.shape
    assert nx % 8 == 0 and ny % 8 == 0 and nz % 8 == 0
    b = occ.reshape(nz // 8, 8, ny // 8, 8, nx // 8, 8)
    b = b.transpose(0, 2, 4, 1, 3, 5)              # bz, by, bx, z, y, x
    any_ = b.reshape(nz // 8, ny // 8, nx // 8, 512).any(axis=3)
    bz, by, bx = np.nonzero(any_)
    xyz = np.stack([bx, by, bz], axis=1).astype(np.int32)
    data = b[bz, by, bx].reshape(-1, 512).astype(np.uint8)
    return np.ascontiguousarray(xyz), np.ascontiguousarray(data)


def blocks_to_dense(xyz: np.ndarray, data: np.ndarray, nx, ny, nz) -> np.ndarray:
    occ = np.zeros((nz, ny, nx), dtype=np.uint8)
    v = occ.reshape(nz // 8, 8, ny // 8, 8, nx // 8, 8)
    for (bx, by, bz), d in zip(xyz, data):
        v[bz, :, by, :, bx, :] = d.reshape(8, 8, 8)
    return occ


# ---------------------------------------------------------------------------
# batched dense maps with room layouts
# ---------------------------------------------------------------------------
def room_layout(rng, nx, ny, nz, min_room=16) -> np.ndarray:
    """Recursive axis-aligned splits into rooms no smaller than `min_room`.
    Each split wall is U{1,2,3} voxels thick and gets one door gap of
    U{3..8} x U{6..12} voxels (clipped to the wall)."""
    occ = np.zeros((nz, ny, nx), dtype=np.uint8)
    stack = [((0, 0, 0), (nx, ny, nz))]
    while stack:
        lo, hi = stack.pop()
        size = [hi[a] - lo[a] for a in range(3)]
        t = int(rng.integers(1, 4))
        cand = [a for a in range(3) if size[a] >= 2 * min_room + t]
        if not cand:
            continue
        w = np.array([size[a] for a in cand], dtype=np.float64)
        a = cand[int(rng.choice(len(cand), p=w / w.sum()))]
        pos = int(rng.integers(lo[a] + min_room, hi[a] - min_room - t + 1))
        o1, o2 = [b for b in range(3) if b != a]
        sl = [slice(lo[b], hi[b]) for b in range(3)]
        sl[a] = slice(pos, pos + t)
        dw = int(rng.integers(3, 9))
        dh = int(rng.integers(6, 13))
        dw, dh = min(dw, size[o1]), min(dh, size[o2])
        d1 = int(rng.integers(lo[o1], hi[o1] - dw + 1))
        d2 = int(rng.integers(lo[o2], hi[o2] - dh + 1))
        occ[sl[2], sl[1], sl[0]] = 1
        gap = list(sl)
        gap[o1] = slice(d1, d1 + dw)
        gap[o2] = slice(d2, d2 + dh)
        occ[gap[2], gap[1], gap[0]] = 0
        hi1 = list(hi); hi1[a] = pos
        lo2 = list(lo); lo2[a] = pos + t
        stack.append((lo, tuple(hi1)))
        stack.append((tuple(lo2), hi))
    return occ


def batch_maps(seed: int, nmaps: int = 64, side_lo: int = 32,
               side_hi: int = 256, rho_lo: float = 0.01, rho_hi: float = 0.30):
    """List of dense uint8 maps (nz, ny, nx); each side U{side_lo..side_hi},
    density U(rho_lo, rho_hi) i.i.d. occupancy unioned with a room layout."""
    rng = np.random.default_rng(seed)
    maps = []
    for _ in range(nmaps):
        nx, ny, nz = (int(rng.integers(side_lo, side_hi + 1)) for _ in range(3))
        rho = float(rng.uniform(rho_lo, rho_hi))
        sub = np.random.default_rng(rng.integers(1 << 62))
        occ = (sub.random((nz, ny, nx), dtype=np.float32) < rho).astype(np.uint8)
        occ |= room_layout(sub, nx, ny, nz)
        maps.append(occ)
    return maps


# ---------------------------------------------------------------------------
# clearance trajectories
# ---------------------------------------------------------------------------
def _bspline_basis(nctrl: int, t: np.ndarray, degree: int = 3) -> np.ndarray:
    """Clamped uniform B-spline basis matrix [len(t), nctrl] (Cox-de Boor)."""
    ninner = nctrl - degree - 1
    knots = np.concatenate([np.zeros(degree + 1),
                            np.arange(1, ninner + 1) / (ninner + 1),
                            np.ones(degree + 1)])
    tt = np.minimum(t, 1.0 - 1e-12)
    nk = len(knots)
    B = np.zeros((len(t), nk - 1))
    for i in range(nk - 1):
        B[:, i] = (knots[i] <= tt) & (tt < knots[i + 1])
    for k in range(1, degree + 1):
        Bn = np.zeros((len(t), nk - 1 - k))
        for i in range(nk - 1 - k):
            a = knots[i + k] - knots[i]
            b = knots[i + k + 1] - knots[i + 1]
            left = (tt - knots[i]) / a * B[:, i] if a > 0 else 0.0
            right = (knots[i + k + 1] - tt) / b * B[:, i + 1] if b > 0 else 0.0
            Bn[:, i] = left + right
        B = Bn
    return B


def trajectories(seed: int, occ: np.ndarray, ntraj: int = 4096,
                 npts: int = 64, nctrl: int = 8, h: float = 0.2) -> np.ndarray:
    """fp32 waypoints [ntraj, npts, 3] as (x, y, z) metres.  Control points are
    drawn uniformly among free voxels of `occ` (voxel center i sits at i*h);
    a clamped uniform cubic B-spline is sampled at npts equally spaced
    parameters, so the end points interpolate the first and last control
    points.  Waypoints may pass through obstacles."""
    rng = np.random.default_rng(seed)
    free = np.flatnonzero(occ.reshape(-1) == 0)
    nz, ny, nx = occ.shape
    pick = free[rng.integers(0, len(free), size=(ntraj, nctrl))]
    x = pick % nx
    y = (pick // nx) % ny
    z = pick // (nx * ny)
    ctrl = np.stack([x, y, z], axis=-1).astype(np.float64) * h  # [T, C, 3]
    B = _bspline_basis(nctrl, np.linspace(0.0, 1.0, npts))        # [W, C]
    wp = np.einsum("wc,tcd->twd", B, ctrl)
    return np.ascontiguousarray(wp.astype(np.float32))
