"""Python binding of libedt: exact truncated squared EDT on an MI355X.

The binding only marshals arguments: every step of the transform runs in the
HIP kernels of ``libedt.so`` (built from ``csrc/`` by ``build.py``).  PyTorch
supplies device memory (the workspace and result tensors) and the stream.
There is no CPU fallback: if the library or a GPU is missing, calls raise.

    f = Field((nx, ny, nz), d_max)
    f.global_(occ)              # occ: torch.uint8 (nz, ny, nx) on the GPU
    f.update(xyz, state)        # xyz: int32 (n, 3) as (x, y, z); state: uint8 (n,)
    s = f.dense()               # int32 (nz, ny, nx): min(d_max^2, squared distance)
    v = f.query(xyz)
    c = ClearanceCost.apply(s, waypoints, h, margin)
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = ["Field", "ClearanceCost", "clearance_cost", "clearance_fwd", "clearance_bwd", "lib",
           "EdtError", "LIB_PATH",
           "Batch", "batch_global", "FUSED", "PER_MAP", "PHASED", "DenseField", "dense_global"]

LIB_PATH = os.environ.get("EDT_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                       "libedt.so")

EDT_OK, EDT_ERR_ARG, EDT_ERR_RANGE, EDT_ERR_CAPACITY, EDT_ERR_HIP, EDT_ERR_STATE = 0, -1, -2, -3, -4, -5
STATUS = {0: "EDT_OK", -1: "EDT_ERR_ARG", -2: "EDT_ERR_RANGE", -3: "EDT_ERR_CAPACITY",
          -4: "EDT_ERR_HIP", -5: "EDT_ERR_STATE"}


class EdtError(RuntimeError):
    def __init__(self, where, code):
        super().__init__(f"{where}: {STATUS.get(code, code)}")
        self.code = code


class EdtConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("d_max", ctypes.c_int32), ("max_blocks", ctypes.c_int64),
                ("max_changes", ctypes.c_int64), ("max_interior_blocks", ctypes.c_int64)]


class EdtMap(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("d_occ", ctypes.c_void_p),
                ("d_block_xyz", ctypes.c_void_p), ("d_block_occ", ctypes.c_void_p),
                ("n_blocks", ctypes.c_int64)]


class EdtStats(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int64), ("obstacle_blocks", ctypes.c_int64),
                ("changed", ctypes.c_int64), ("added", ctypes.c_int64),
                ("removed", ctypes.c_int64), ("seed_blocks", ctypes.c_int64),
                ("raise_blocks", ctypes.c_int64), ("lower_blocks", ctypes.c_int64),
                ("dirty_blocks", ctypes.c_int64), ("error", ctypes.c_int32),
                ("d_max", ctypes.c_int32)]


class EdtBatchMap(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("occ_offset", ctypes.c_int64),
                ("out_offset", ctypes.c_int64)]


class EdtTune(ctypes.Structure):
    _fields_ = [("lrun", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("wg_waves", ctypes.c_int32)]


_lib = None


def lib():
    """Load libedt.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2105_04419_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
    f64 = ctypes.c_double
    sig = {
        "edt_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "edt_workspace_bytes": ([ctypes.POINTER(EdtConfig)], i64),
        "edt_create": ([ctypes.POINTER(EdtConfig), vp, i64, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "edt_destroy": ([vp], ctypes.c_int),
        "edt_global": ([vp, ctypes.POINTER(EdtMap), vp], ctypes.c_int),
        "edt_update": ([vp, vp, vp, i64, vp], ctypes.c_int),
        "edt_query": ([vp, vp, i64, vp, vp], ctypes.c_int),
        "edt_query_nearest": ([vp, vp, i64, vp, vp], ctypes.c_int),
        "edt_compact": ([vp, vp], ctypes.c_int),
        "edt_grow": ([vp, i64, vp, i64, vp], ctypes.c_int),
        "edt_integrate_scan": ([vp, vp, vp, vp, i64, vp], ctypes.c_int),
        "edt_interior": ([vp, vp], ctypes.c_int),
        "edt_query_signed": ([vp, vp, i64, vp, vp], ctypes.c_int),
        "edt_read_signed_dense": ([vp, vp, vp], ctypes.c_int),
        "edt_read_dense": ([vp, vp, vp], ctypes.c_int),
        "edt_read_occupancy": ([vp, vp, vp], ctypes.c_int),
        "edt_get_stats": ([vp, ctypes.POINTER(EdtStats), vp], ctypes.c_int),
        "edt_get_error": ([vp, vp], ctypes.c_int),
        "edt_timing_begin": ([vp, i32], ctypes.c_int),
        "edt_timing_begin_phase": ([vp, i32, i32], ctypes.c_int),
        "edt_timing_read": ([vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i32)],
                            ctypes.c_int),
        "edt_batch_workspace_bytes": ([ctypes.POINTER(EdtBatchMap), i32, i32], i64),
        "edt_batch_create": ([ctypes.POINTER(EdtBatchMap), i32, i32, vp, i64, vp,
                              ctypes.POINTER(vp)], ctypes.c_int),
        "edt_batch_run": ([vp, vp, vp, i32, ctypes.POINTER(EdtTune), vp], ctypes.c_int),
        "edt_batch_destroy": ([vp], ctypes.c_int),
        "edt_dense_workspace_bytes": ([i32, i32, i32], i64),
        "edt_dense_global": ([i32, i32, i32, i32, vp, vp, vp, i64, vp], ctypes.c_int),
        "edt_dense_global_noalloc": ([i32, i32, i32, i32, vp, vp, vp], ctypes.c_int),
        "edt_dense_ctx_bytes": ([i32, i32, i32, i64], i64),
        "edt_dense_ctx_create": ([i32, i32, i32, i32, i64, vp, i64, vp, ctypes.POINTER(vp)],
                                 ctypes.c_int),
        "edt_dense_ctx_destroy": ([vp], ctypes.c_int),
        "edt_dense_ctx_global": ([vp, vp, vp], ctypes.c_int),
        "edt_dense_ctx_update": ([vp, vp, vp, i64, vp], ctypes.c_int),
        "edt_dense_ctx_field": ([vp], vp),
        "edt_dense_ctx_get_error": ([vp, vp], ctypes.c_int),
        "edt_clearance_fwd": ([vp, i32, i32, i32, f64, f32, vp, i64, i32, vp, vp], ctypes.c_int),
        "edt_clearance_bwd": ([vp, i32, i32, i32, f64, f32, vp, i64, i32, vp, vp, vp],
                              ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return _lib


def _check(where, rc):
    if rc != EDT_OK:
        raise EdtError(where, rc)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev_tensor(t, dtype, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.contiguous()


class Field:
    """Distance field of one voxel map: a context of libedt plus its
    workspace (a torch uint8 tensor that owns the device memory)."""

    def __init__(self, shape, d_max: int, max_blocks: int = 0, max_changes: int = 0,
                 max_interior_blocks: int = 0, device=None, stream=None):
        nx, ny, nz = (int(v) for v in shape)
        self.shape = (nx, ny, nz)
        self.d_max = int(d_max)
        self.D = self.d_max * self.d_max
        self.cfg = EdtConfig(nx, ny, nz, self.d_max, int(max_blocks), int(max_changes),
                             int(max_interior_blocks))
        L = lib()
        nbytes = L.edt_workspace_bytes(ctypes.byref(self.cfg))
        if nbytes < 0:
            raise EdtError("edt_workspace_bytes", int(nbytes))
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        nb = ((nx + 7) // 8) * ((ny + 7) // 8) * ((nz + 7) // 8)
        self.extent_blocks = nb
        self.max_blocks = min(int(max_blocks), nb) if max_blocks else nb
        ctx = ctypes.c_void_p()
        _check("edt_create", L.edt_create(ctypes.byref(self.cfg), _ptr(self.workspace),
                                          int(nbytes), _stream(stream), ctypes.byref(ctx)))
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            lib().edt_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- transforms ---------------------------------------------------------
    def _grown(self, call, grow: bool, stream):
        """Run call(); with grow, wait for it and, while the device reports a
        full pool (the call was cancelled with the map unchanged, or a global
        transform ran out of room), double the pool and run it again."""
        call()
        while grow:
            err = self.error(stream)
            if err != EDT_ERR_CAPACITY or self.max_blocks >= self.extent_blocks:
                if err != EDT_OK:
                    raise EdtError("device error", err)
                break
            self.grow(min(2 * self.max_blocks, self.extent_blocks), stream)
            call()
        return self

    def global_(self, occ: torch.Tensor, stream=None, grow: bool = False):
        """Global transform of a dense occupancy grid (nz, ny, nx) uint8.
        grow: enlarge the pool until the map fits (waits for the GPU)."""
        nx, ny, nz = self.shape
        occ = _dev_tensor(occ, torch.uint8, (nz, ny, nx))
        m = EdtMap(0, occ.data_ptr(), None, None, 0)
        self._keep = occ
        return self._grown(lambda: _check("edt_global", lib().edt_global(
            self._ctx, ctypes.byref(m), _stream(stream))), grow, stream)

    def global_blocks(self, block_xyz: torch.Tensor, block_occ: torch.Tensor, stream=None,
                      grow: bool = False):
        """Global transform of a leaf-block list: block_xyz int32 (n, 3) as
        (bx, by, bz), block_occ uint8 (n, 512) with in-block index x+8y+64z."""
        n = int(block_xyz.shape[0])
        xyz = _dev_tensor(block_xyz, torch.int32, (n, 3))
        data = _dev_tensor(block_occ, torch.uint8, (n, 512))
        m = EdtMap(1, None, xyz.data_ptr() if n else None, data.data_ptr() if n else None, n)
        self._keep = (xyz, data)
        return self._grown(lambda: _check("edt_global", lib().edt_global(
            self._ctx, ctypes.byref(m), _stream(stream))), grow, stream)

    def update(self, xyz: torch.Tensor, state: torch.Tensor, stream=None, grow: bool = False):
        """Incremental transform: set voxels xyz (int32 (n, 3)) to the
        absolute occupancy `state` (uint8 (n,)); the last entry wins.
        grow: if the pool is full, enlarge it and repeat the (cancelled)
        update (waits for the GPU)."""
        n = int(xyz.shape[0])
        if n == 0:
            return self
        xyz = _dev_tensor(xyz, torch.int32, (n, 3))
        state = _dev_tensor(state, torch.uint8, (n,))
        self._keep = (xyz, state)
        return self._grown(lambda: _check("edt_update", lib().edt_update(
            self._ctx, _ptr(xyz), _ptr(state), n, _stream(stream))), grow, stream)

    def grow(self, max_blocks: int | None = None, stream=None):
        """Move the field onto a larger block pool (edt_grow): max_blocks
        slots (default: twice the current pool, at most one per block of the
        extent).  The map and field carry over unchanged."""
        new = int(max_blocks) if max_blocks else min(2 * self.max_blocks, self.extent_blocks)
        new = min(new, self.extent_blocks)
        cfg = EdtConfig(self.cfg.nx, self.cfg.ny, self.cfg.nz, self.cfg.d_max, new,
                        self.cfg.max_changes, self.cfg.max_interior_blocks)
        L = lib()
        nbytes = L.edt_workspace_bytes(ctypes.byref(cfg))
        if nbytes < 0:
            raise EdtError("edt_workspace_bytes", int(nbytes))
        ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        _check("edt_grow", L.edt_grow(self._ctx, new, _ptr(ws), int(nbytes), _stream(stream)))
        if stream is not None:
            # the old workspace is read by the work just enqueued on `stream`
            self.workspace.record_stream(stream)
        self.workspace, self.cfg, self.max_blocks = ws, cfg, new
        return self

    def integrate_scan(self, origin: torch.Tensor, ends: torch.Tensor, hits: torch.Tensor,
                       stream=None):
        """Integrate one range scan (sensor voxel origin int32 (3,), ray end
        voxels int32 (n, 3), hits uint8 (n,)) into the occupancy and update
        the field incrementally."""
        n = int(ends.shape[0])
        if n == 0:
            return self
        origin = _dev_tensor(origin, torch.int32, (3,))
        ends = _dev_tensor(ends, torch.int32, (n, 3))
        hits = _dev_tensor(hits, torch.uint8, (n,))
        _check("edt_integrate_scan", lib().edt_integrate_scan(self._ctx, _ptr(origin), _ptr(ends),
                                                              _ptr(hits), n, _stream(stream)))
        self._keep = (origin, ends, hits)
        return self

    def compact(self, stream=None):
        """Rebuild the block pool from the current occupancy (drops blocks no
        longer within reach of an obstacle); the field is unchanged."""
        _check("edt_compact", lib().edt_compact(self._ctx, _stream(stream)))
        return self

    # -- reads ----------------------------------------------------------------
    def query(self, xyz: torch.Tensor, stream=None) -> torch.Tensor:
        n = int(xyz.shape[0])
        out = torch.empty(n, dtype=torch.int32, device=self.device)
        if n:
            xyz = _dev_tensor(xyz, torch.int32, (n, 3))
            _check("edt_query", lib().edt_query(self._ctx, _ptr(xyz), n, _ptr(out),
                                                _stream(stream)))
        return out

    def query_nearest(self, xyz: torch.Tensor, stream=None) -> torch.Tensor:
        """Coordinates (x, y, z) of one nearest obstacle per query voxel,
        (-1, -1, -1) where none lies within d_max."""
        n = int(xyz.shape[0])
        out = torch.empty((n, 3), dtype=torch.int32, device=self.device)
        if n:
            xyz = _dev_tensor(xyz, torch.int32, (n, 3))
            _check("edt_query_nearest", lib().edt_query_nearest(self._ctx, _ptr(xyz), n, _ptr(out),
                                                                _stream(stream)))
        return out

    def interior(self, stream=None):
        """Interior distances of the occupied voxels (squared distance to the
        nearest free voxel, clamped to D), valid until the next transform."""
        _check("edt_interior", lib().edt_interior(self._ctx, _stream(stream)))
        return self

    def query_signed(self, xyz: torch.Tensor, stream=None) -> torch.Tensor:
        """Signed squared distances: s on free voxels, -(interior) on occupied ones."""
        n = int(xyz.shape[0])
        out = torch.empty(n, dtype=torch.int32, device=self.device)
        xyz = _dev_tensor(xyz, torch.int32, (n, 3)) if n else xyz
        _check("edt_query_signed", lib().edt_query_signed(self._ctx, _ptr(xyz) if n else None, n,
                                                          _ptr(out) if n else None,
                                                          _stream(stream)))
        return out

    def signed_dense(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        nx, ny, nz = self.shape
        if out is None:
            out = torch.empty((nz, ny, nx), dtype=torch.int32, device=self.device)
        out = _dev_tensor(out, torch.int32, (nz, ny, nx))
        _check("edt_read_signed_dense", lib().edt_read_signed_dense(self._ctx, _ptr(out),
                                                                    _stream(stream)))
        return out

    def dense(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        nx, ny, nz = self.shape
        if out is None:
            out = torch.empty((nz, ny, nx), dtype=torch.int32, device=self.device)
        out = _dev_tensor(out, torch.int32, (nz, ny, nx))
        _check("edt_read_dense", lib().edt_read_dense(self._ctx, _ptr(out), _stream(stream)))
        return out

    def occupancy(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        nx, ny, nz = self.shape
        if out is None:
            out = torch.empty((nz, ny, nx), dtype=torch.uint8, device=self.device)
        out = _dev_tensor(out, torch.uint8, (nz, ny, nx))
        _check("edt_read_occupancy", lib().edt_read_occupancy(self._ctx, _ptr(out), _stream(stream)))
        return out

    def stats(self, stream=None) -> dict:
        st = EdtStats()
        _check("edt_get_stats", lib().edt_get_stats(self._ctx, ctypes.byref(st), _stream(stream)))
        return {k: getattr(st, k) for k, _ in EdtStats._fields_}

    PHASES = ("ingest", "region", "items", "pass_x", "pass_y", "pass_z")

    def timing_begin(self, n_calls: int, phase: str | None = None):
        """Record HIP events around the phases of the next n_calls global
        transforms (profiling); with `phase` (one of PHASES) only that phase
        is bracketed."""
        k = -1 if phase is None else self.PHASES.index(phase)
        _check("edt_timing_begin_phase",
               lib().edt_timing_begin_phase(self._ctx, int(n_calls), k))

    def timing_read(self) -> dict:
        """Mean phase durations (ms) over the recorded calls."""
        ms = (ctypes.c_float * 6)()
        n = ctypes.c_int32()
        _check("edt_timing_read", lib().edt_timing_read(self._ctx, ms, ctypes.byref(n)))
        d = {k: float(ms[i]) for i, k in enumerate(self.PHASES)}
        d["calls"] = int(n.value)
        return d

    def error(self, stream=None) -> int:
        """Device error word (0 or a negative status); reading clears it."""
        return int(lib().edt_get_error(self._ctx, _stream(stream)))


# ---------------------------------------------------------------------------
# full (uncapped) transform of a dense grid
# ---------------------------------------------------------------------------
DENSE_INF = 0x7fffffff


def dense_global(occ: torch.Tensor, d_max: int = 0, out: torch.Tensor | None = None,
                 workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Exact squared EDT of a dense grid occ (nz, ny, nx) uint8 with no
    radius (d_max = 0; voxels of a grid without obstacles get DENSE_INF) or
    clamped to d_max^2.  Returns int32 (nz, ny, nx)."""
    nz, ny, nx = (int(v) for v in occ.shape)
    occ = _dev_tensor(occ, torch.uint8, (nz, ny, nx))
    L = lib()
    nbytes = int(L.edt_dense_workspace_bytes(nx, ny, nz))
    if nbytes < 0:
        raise EdtError("edt_dense_workspace_bytes", nbytes)
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.int32, device=occ.device)
    out = _dev_tensor(out, torch.int32, (nz, ny, nx))
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=occ.device)
    _check("edt_dense_global", L.edt_dense_global(nx, ny, nz, int(d_max), _ptr(occ), _ptr(out),
                                                  _ptr(workspace), workspace.numel(),
                                                  _stream(stream)))
    return out


DENSE_STATIC_BYTES = 64 << 20


class DenseField:
    """Uncapped (d_max = 0) or large-radius field of a dense grid kept
    current under occupancy changes (edt_dense_ctx_*): global transform,
    incremental updates, and the int32 field as a view of the workspace."""

    def __init__(self, shape, d_max: int = 0, max_changes: int = 1 << 20, device=None,
                 stream=None):
        nx, ny, nz = (int(v) for v in shape)
        self.shape = (nx, ny, nz)
        self.d_max = int(d_max)
        L = lib()
        nbytes = int(L.edt_dense_ctx_bytes(nx, ny, nz, int(max_changes)))
        if nbytes < 0:
            raise EdtError("edt_dense_ctx_bytes", nbytes)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        _check("edt_dense_ctx_create", L.edt_dense_ctx_create(
            nx, ny, nz, self.d_max, int(max_changes), _ptr(self.workspace), nbytes,
            _stream(stream), ctypes.byref(ctx)))
        self._ctx = ctx
        off = int(L.edt_dense_ctx_field(ctx)) - self.workspace.data_ptr()
        n = nx * ny * nz
        self._field = self.workspace[off:off + 4 * n].view(torch.int32).view(nz, ny, nx)

    def close(self):
        if getattr(self, "_ctx", None):
            lib().edt_dense_ctx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def global_(self, occ: torch.Tensor, stream=None):
        nx, ny, nz = self.shape
        occ = _dev_tensor(occ, torch.uint8, (nz, ny, nx))
        _check("edt_dense_ctx_global", lib().edt_dense_ctx_global(self._ctx, _ptr(occ),
                                                                   _stream(stream)))
        self._keep = occ
        return self

    def update(self, xyz: torch.Tensor, state: torch.Tensor, stream=None):
        """Set voxels xyz (int32 (n, 3)) to the absolute occupancy `state`
        (uint8 (n,)); the last entry of a voxel wins."""
        n = int(xyz.shape[0])
        if n == 0:
            return self
        xyz = _dev_tensor(xyz, torch.int32, (n, 3))
        state = _dev_tensor(state, torch.uint8, (n,))
        _check("edt_dense_ctx_update", lib().edt_dense_ctx_update(
            self._ctx, _ptr(xyz), _ptr(state), n, _stream(stream)))
        self._keep = (xyz, state)
        return self

    def field(self) -> torch.Tensor:
        """The int32 field (nz, ny, nx): a view of the workspace, current once
        the work enqueued before has completed."""
        return self._field

    def error(self, stream=None) -> int:
        return int(lib().edt_dense_ctx_get_error(self._ctx, _stream(stream)))


def dense_global_noalloc(occ: torch.Tensor, d_max: int = 0, out: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
    """dense_global without a workspace (edt_dense_global_noalloc): the
    library's static per-GPU buffer holds the envelopes, so grids are limited
    to DENSE_STATIC_BYTES / 8 voxels.  Calls that overlap on one GPU race.
    With `out` given, the call itself allocates nothing."""
    nz, ny, nx = (int(v) for v in occ.shape)
    occ = _dev_tensor(occ, torch.uint8, (nz, ny, nx))
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.int32, device=occ.device)
    out = _dev_tensor(out, torch.int32, (nz, ny, nx))
    _check("edt_dense_global_noalloc",
           lib().edt_dense_global_noalloc(nx, ny, nz, int(d_max), _ptr(occ), _ptr(out),
                                          _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# clearance cost
# ---------------------------------------------------------------------------
def _clearance_args(s, wp):
    if s.dim() != 3:
        raise ValueError("field must be (nz, ny, nx)")
    s = _dev_tensor(s, torch.int32)
    wp = _dev_tensor(wp, torch.float32)
    if wp.dim() != 3 or wp.shape[-1] != 3:
        raise ValueError("waypoints must be (T, W, 3)")
    nz, ny, nx = s.shape
    return s, wp, nx, ny, nz


def clearance_fwd(s, wp, h: float, margin: float, out=None, stream=None):
    """edt_clearance_fwd: per-trajectory cost (float32 [T]) of waypoints
    wp (T, W, 3) on the int32 field s (nz, ny, nx), no autograd."""
    s, wp, nx, ny, nz = _clearance_args(s, wp)
    T, W = int(wp.shape[0]), int(wp.shape[1])
    if out is None:
        out = torch.empty(T, dtype=torch.float32, device=wp.device)
    out = _dev_tensor(out, torch.float32, (T,))
    _check("edt_clearance_fwd", lib().edt_clearance_fwd(
        _ptr(s), nx, ny, nz, float(h), float(margin), _ptr(wp), T, W, _ptr(out), _stream(stream)))
    return out


def clearance_bwd(s, wp, gcost, h: float, margin: float, out=None, stream=None):
    """edt_clearance_bwd: gcost[t] * d C[t] / d wp (float32 (T, W, 3))."""
    s, wp, nx, ny, nz = _clearance_args(s, wp)
    T, W = int(wp.shape[0]), int(wp.shape[1])
    gcost = _dev_tensor(gcost.to(torch.float32), torch.float32, (T,))
    if out is None:
        out = torch.empty_like(wp)
    out = _dev_tensor(out, torch.float32, tuple(wp.shape))
    _check("edt_clearance_bwd", lib().edt_clearance_bwd(
        _ptr(s), nx, ny, nz, float(h), float(margin), _ptr(wp), T, W, _ptr(gcost), _ptr(out),
        _stream(stream)))
    return out


class ClearanceCost(torch.autograd.Function):
    """C[t] = sum_w max(0, margin - d(wp[t, w]))^2 with d the trilinear
    interpolant of h*sqrt(s); forward and backward are HIP kernels."""

    @staticmethod
    def forward(ctx, s, wp, h: float, margin: float):
        s = _dev_tensor(s, torch.int32)
        wp = _dev_tensor(wp, torch.float32)
        cost = clearance_fwd(s, wp, h, margin)
        ctx.save_for_backward(s, wp)
        ctx.h, ctx.margin = float(h), float(margin)
        return cost

    @staticmethod
    def backward(ctx, gcost):
        s, wp = ctx.saved_tensors
        return None, clearance_bwd(s, wp, gcost.contiguous(), ctx.h, ctx.margin), None, None


def clearance_cost(s, wp, h: float = 0.2, margin: float = 1.0):
    return ClearanceCost.apply(s, wp, h, margin)


# ---------------------------------------------------------------------------
# batched dense maps
# ---------------------------------------------------------------------------
FUSED, PER_MAP, PHASED = 0, 1, 2
DEFAULT_TUNE = {"lrun": 8, "waves_per_cu": 8, "chunk": 4, "schedule": 0, "wg_waves": 4}


class Batch:
    """Many dense maps transformed together.  Occupancy of all maps lives in
    one flat uint8 tensor, the fields in one flat int32 tensor; map i uses
    the slice [offsets[i], offsets[i] + nx*ny*nz) of both (grid layout, x
    fastest)."""

    def __init__(self, shapes, d_max: int, device=None, stream=None):
        self.shapes = [tuple(int(v) for v in sh) for sh in shapes]   # (nx, ny, nz)
        self.d_max = int(d_max)
        self.offsets = []
        off = 0
        for nx, ny, nz in self.shapes:
            self.offsets.append(off)
            off += nx * ny * nz
        self.total = off
        n = len(self.shapes)
        self._maps = (EdtBatchMap * n)(*[EdtBatchMap(nx, ny, nz, 0, o, o) for (nx, ny, nz), o
                                         in zip(self.shapes, self.offsets)])
        L = lib()
        nbytes = L.edt_batch_workspace_bytes(self._maps, n, self.d_max)
        if nbytes < 0:
            raise EdtError("edt_batch_workspace_bytes", int(nbytes))
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check("edt_batch_create", L.edt_batch_create(self._maps, n, self.d_max, _ptr(self.workspace),
                                                      int(nbytes), _stream(stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().edt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, maps) -> torch.Tensor:
        """Concatenate per-map (nz, ny, nx) uint8 arrays into the flat input."""
        flat = torch.empty(self.total, dtype=torch.uint8, device=self.device)
        for m, o, (nx, ny, nz) in zip(maps, self.offsets, self.shapes):
            t = m if isinstance(m, torch.Tensor) else torch.from_numpy(m)
            flat[o:o + nx * ny * nz] = t.reshape(-1).to(self.device)
        return flat

    def unpack(self, out: torch.Tensor):
        return [out[o:o + nx * ny * nz].view(nz, ny, nx)
                for o, (nx, ny, nz) in zip(self.offsets, self.shapes)]

    def run(self, occ_flat: torch.Tensor, out: torch.Tensor | None = None, mode: int | None = None,
            tune: dict | None = None, stream=None) -> torch.Tensor:
        """mode: FUSED, PHASED or PER_MAP; None takes the schedule's "mode"
        entry (as the autotuner returns it), else FUSED."""
        if mode is None:
            mode = (tune or {}).get("mode", FUSED)
        occ_flat = _dev_tensor(occ_flat, torch.uint8, (self.total,))
        if out is None:
            out = torch.empty(self.total, dtype=torch.int32, device=self.device)
        out = _dev_tensor(out, torch.int32, (self.total,))
        t = dict(DEFAULT_TUNE)
        if tune:
            t.update(tune)
        tt = EdtTune(t["lrun"], t["waves_per_cu"], t["chunk"], t["schedule"], t["wg_waves"])
        _check("edt_batch_run", lib().edt_batch_run(self._h, _ptr(occ_flat), _ptr(out), int(mode),
                                                    ctypes.byref(tt), _stream(stream)))
        return out


def batch_global(maps, d_max: int, mode: int | None = None, tune: dict | None = None):
    """Transform a list of dense (nz, ny, nx) uint8 maps; returns int32 fields."""
    shapes = [(m.shape[2], m.shape[1], m.shape[0]) for m in maps]
    b = Batch(shapes, d_max)
    out = b.run(b.pack(maps), mode=mode, tune=tune)
    return b.unpack(out)
