"""CPU oracle -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library
(``paper_2105_04419_amd``) never imports it and shares no code with it.

Contents
  edt_bruteforce / edt_points / edt_separable
      The truncated squared Euclidean distance transform of the VDB-EDT paper
      (section III, Eq. 1, limited to the transform radius d_max), written in
      plain C in ``edt_oracle.c`` and called through ctypes.
  edt_points_list
      The same definition for an obstacle list (sparse maps on huge extents).
  edt_uncapped
      The definition without a radius (the full transform).
  interior / signed_field
      The inside half of a signed distance field: the same definition with
      occupied and free voxels exchanged (the squared distance from an
      occupied voxel to the nearest free voxel of the extent, clamped to D),
      and the signed field that combines the two.
  Alg1
      The paper's Algorithm 1 itself on the CPU (``alg1.c``), to measure what
      its procedure computes and costs; not an oracle.
  ray_voxels / integrate_scan
      The occupancy integration of a range scan in front of the transform
      (``scan_oracle.c``): the exact integer voxel walk of a ray and the
      free / hit marking of one scan.
  clearance (module ``oracle.clearance``)
      The trajectory clearance cost built on the distance field (section III,
      Eq. 2 clearance term, squared hinge form), its analytic gradient and a
      central finite-difference gradient, all in float64 numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "edt_oracle.c")
_SRC_SCAN = os.path.join(_HERE, "scan_oracle.c")
_SRC_ALG1 = os.path.join(_HERE, "alg1.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile edt_oracle.c and scan_oracle.c with gcc (-O2, OpenMP) into
    oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                        "-Wall", "-o", tmp, _SRC, _SRC_SCAN, _SRC_ALG1], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        ci = ctypes.c_int
        L.oracle_edt_bruteforce.argtypes = [u8p, ci, ci, ci, ci, i32p]
        L.oracle_edt_points.argtypes = [u8p, ci, ci, ci, ci, i32p, ctypes.c_int64, i32p]
        L.oracle_edt_separable.argtypes = [u8p, ci, ci, ci, ci, i32p]
        L.oracle_threads.argtypes = [ci]
        L.oracle_ray_voxels.argtypes = [i32p, i32p, i32p, ctypes.c_int64]
        L.oracle_ray_voxels.restype = ctypes.c_int64
        L.oracle_integrate_scan.argtypes = [u8p, ci, ci, ci, i32p, i32p, u8p, ctypes.c_int64]
        L.oracle_integrate_scan.restype = ctypes.c_int64
        vp = ctypes.c_void_p
        L.alg1_create.argtypes = [ci, ci, ci, ci, ci]
        L.alg1_create.restype = vp
        L.alg1_destroy.argtypes = [vp]
        L.alg1_destroy.restype = None
        L.alg1_apply.argtypes = [vp, i32p, u8p, ctypes.c_int64]
        L.alg1_apply.restype = None
        L.alg1_transform.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.alg1_transform.restype = None
        L.alg1_read.argtypes = [vp, i32p]
        L.alg1_read.restype = None
        for f in (L.oracle_edt_bruteforce, L.oracle_edt_points,
                  L.oracle_edt_separable, L.oracle_threads):
            f.restype = ci
        _lib = L
    return _lib


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _grid(occ):
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    assert occ.ndim == 3
    nz, ny, nx = occ.shape
    return occ, nx, ny, nz


def edt_bruteforce(occ: np.ndarray, dmax: int) -> np.ndarray:
    """s = min(D, min_y |x-y|^2) for every voxel; occ is (nz, ny, nx)."""
    occ, nx, ny, nz = _grid(occ)
    out = np.empty(occ.shape, dtype=np.int32)
    rc = lib().oracle_edt_bruteforce(_u8(occ), nx, ny, nz, int(dmax), _i32(out))
    if rc:
        raise ValueError(f"oracle_edt_bruteforce: bad arguments ({rc})")
    return out


def edt_points(occ: np.ndarray, dmax: int, xyz: np.ndarray) -> np.ndarray:
    """The definition evaluated at voxels xyz int[n, 3] given as (x, y, z)."""
    occ, nx, ny, nz = _grid(occ)
    xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
    out = np.empty(len(xyz), dtype=np.int32)
    rc = lib().oracle_edt_points(_u8(occ), nx, ny, nz, int(dmax), _i32(xyz),
                                 len(xyz), _i32(out))
    if rc:
        raise ValueError(f"oracle_edt_points: bad arguments ({rc})")
    return out


def edt_separable(occ: np.ndarray, dmax: int) -> np.ndarray:
    """Same field as edt_bruteforce, one axis at a time (fast enough for
    the 1024x1024x128 extent)."""
    occ, nx, ny, nz = _grid(occ)
    out = np.empty(occ.shape, dtype=np.int32)
    rc = lib().oracle_edt_separable(_u8(occ), nx, ny, nz, int(dmax), _i32(out))
    if rc:
        raise ValueError(f"oracle_edt_separable: failed ({rc})")
    return out


def edt_points_list(obstacles: np.ndarray, dmax: int, xyz: np.ndarray) -> np.ndarray:
    """Eq. 1 at voxels xyz (int[n, 3], (x, y, z)) for an obstacle set given
    as a list of voxel coordinates (int[m, 3]) instead of a grid: for sparse
    maps on extents far too large to hold densely.  Plain all-pairs minimum
    (numpy, in chunks)."""
    obs = np.asarray(obstacles, dtype=np.int64).reshape(-1, 3)
    q = np.asarray(xyz, dtype=np.int64).reshape(-1, 3)
    D = int(dmax) * int(dmax)
    out = np.full(len(q), D, dtype=np.int64)
    if len(obs) == 0:
        return out.astype(np.int32)
    step = max(1, (1 << 22) // len(obs))
    for i in range(0, len(q), step):
        d2 = ((q[i:i + step, None, :] - obs[None, :, :]) ** 2).sum(-1).min(1)
        out[i:i + step] = np.minimum(d2, D)
    return out.astype(np.int32)


INF = 0x7FFFFFFF


def edt_uncapped(occ: np.ndarray) -> np.ndarray:
    """Eq. 1 with no radius: the exact squared distance to the nearest
    obstacle (INF on a grid without obstacles).  A radius beyond the grid's
    diagonal never clamps, so this is edt_separable at such a radius."""
    occ, nx, ny, nz = _grid(occ)
    if not occ.any():
        return np.full(occ.shape, INF, dtype=np.int32)
    r = int(np.ceil(np.sqrt(float(nx) ** 2 + float(ny) ** 2 + float(nz) ** 2))) + 1
    if r > 4095:
        raise ValueError("edt_uncapped: grid too large for the windowed oracle")
    return edt_separable(occ, r)


def interior(occ: np.ndarray, dmax: int) -> np.ndarray:
    """min(D, min over free voxels y of |x-y|^2) for every voxel: Eq. 1 on
    the complement of the occupancy.  Voxels outside the extent are neither
    free nor occupied, so a voxel with no free voxel within d_max gets D."""
    occ, _, _, _ = _grid(occ)
    return edt_separable((occ == 0).astype(np.uint8), dmax)


def signed_field(occ: np.ndarray, dmax: int) -> np.ndarray:
    """Signed squared distance: s(x) on free voxels, -interior(x) on
    occupied voxels (so 0 never occurs: s >= 1 off obstacles, interior >= 1
    on them)."""
    occ, _, _, _ = _grid(occ)
    return np.where(occ != 0, -interior(occ, dmax), edt_separable(occ, dmax)).astype(np.int32)


def ray_voxels(o, e) -> np.ndarray:
    """Voxels (x, y, z) visited by the ray from voxel o to voxel e, in walk
    order (scan_oracle.c states the traversal rule)."""
    o = np.ascontiguousarray(o, dtype=np.int32)
    e = np.ascontiguousarray(e, dtype=np.int32)
    n = int(np.abs(e.astype(np.int64) - o).sum()) + 1
    out = np.empty((n, 3), dtype=np.int32)
    got = lib().oracle_ray_voxels(_i32(o), _i32(e), _i32(out), n)
    assert got == n
    return out


def integrate_scan(occ: np.ndarray, origin, ends: np.ndarray, hits: np.ndarray):
    """One scan integrated into a copy of occ (nz, ny, nx): visited voxels
    free, hit end voxels occupied (hits win).  Returns (new occupancy, number
    of rays skipped for an endpoint outside the grid)."""
    occ, nx, ny, nz = _grid(occ)
    occ = occ.copy()
    o = np.ascontiguousarray(origin, dtype=np.int32).reshape(3)
    e = np.ascontiguousarray(ends, dtype=np.int32).reshape(-1, 3)
    h = np.ascontiguousarray(hits, dtype=np.uint8).reshape(-1)
    assert len(e) == len(h)
    sk = lib().oracle_integrate_scan(_u8(occ), nx, ny, nz, _i32(o), _i32(e), _u8(h), len(e))
    if sk < 0:
        raise ValueError("oracle_integrate_scan: bad arguments")
    return occ, int(sk)


class Alg1:
    """The paper's Algorithm 1 on the CPU (``alg1.c``): SetObstacle /
    RemoveObstacle, then DistanceTransform with raising and lowering waves
    over the 26-neighbourhood.  schedule "transform_status" is the paper's
    method (section IV-B: the raise key is the transform radius, and a
    lowering wave may take over a raising front); "conventional" is the
    scheme it improves on (a raise flag, raising fronts are never taken
    over).  Not an oracle: it is the paper's own procedure, whose result the
    tests compare with the exact field."""

    SCHEDULES = {"conventional": 0, "transform_status": 1}

    def __init__(self, shape, dmax: int, schedule: str = "transform_status"):
        nx, ny, nz = (int(v) for v in shape)
        self.shape = (nx, ny, nz)
        self.schedule = schedule
        self._h = lib().alg1_create(nx, ny, nz, int(dmax), self.SCHEDULES[schedule])
        if not self._h:
            raise ValueError("alg1_create failed")

    def close(self):
        if getattr(self, "_h", None):
            lib().alg1_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def apply(self, xyz, state):
        xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
        state = np.ascontiguousarray(state, dtype=np.uint8).reshape(-1)
        lib().alg1_apply(self._h, _i32(xyz), _u8(state), len(xyz))
        return self

    def set_map(self, occ):
        """SetObstacle for every occupied voxel of occ (nz, ny, nx)."""
        xyz = np.argwhere(np.asarray(occ) != 0)[:, ::-1]
        return self.apply(xyz, np.ones(len(xyz), np.uint8))

    def transform(self):
        """DistanceTransform; returns (fronts lowered, fronts raised)."""
        c = (ctypes.c_int64 * 2)()
        lib().alg1_transform(self._h, c)
        return int(c[0]), int(c[1])

    def field(self) -> np.ndarray:
        nx, ny, nz = self.shape
        out = np.empty((nz, ny, nx), dtype=np.int32)
        lib().alg1_read(self._h, _i32(out))
        return out


def threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count of the oracle."""
    return int(lib().oracle_threads(int(n)))
