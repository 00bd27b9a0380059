"""The allocation-free dense transform (edt_dense_global_noalloc) against the
workspace form (edt_dense_global), both called through the C ABI: two calls
in a row, the second on a smaller grid, must give the same int32 fields bit
for bit (and the oracle's on the small grid); a grid beyond the static
buffer is refused with nothing written."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2105_04419_amd import DENSE_STATIC_BYTES, lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    oracle.build(force=False)


def vp(t):
    return ctypes.c_void_p(t.data_ptr())


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def call_noalloc(occ, d_max):
    nz, ny, nx = occ.shape
    out = torch.full((nz, ny, nx), -7, dtype=torch.int32, device="cuda")
    rc = lib().edt_dense_global_noalloc(nx, ny, nz, d_max, vp(occ), vp(out), stream())
    assert rc == 0, rc
    return out


def call_workspace(occ, d_max):
    nz, ny, nx = occ.shape
    L = lib()
    nbytes = int(L.edt_dense_workspace_bytes(nx, ny, nz))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = torch.full((nz, ny, nx), -9, dtype=torch.int32, device="cuda")
    rc = L.edt_dense_global(nx, ny, nz, d_max, vp(occ), vp(out), vp(ws), nbytes, stream())
    assert rc == 0, rc
    return out


def grid(seed, shape, p):
    rng = np.random.default_rng(seed)
    return (rng.random(shape) < p).astype(np.uint8)


@pytest.mark.parametrize("d_max", [0, 40])
def test_two_calls_second_smaller(d_max):
    # the largest grid the static buffer holds (256 x 256 x 128 voxels, 8 B of
    # envelope each), then a small ragged one: the second call must not see
    # anything of the first in the shared buffer
    big = np.zeros((128, 256, 256), np.uint8)
    big[::37, ::41, ::29] = 1
    big[60:70, 100:140, 30:34] = 1
    assert big.size * 8 == DENSE_STATIC_BYTES
    small = grid(3, (23, 29, 37), 0.01)
    outs = []
    for occ in (big, small):
        occ_d = torch.from_numpy(occ).cuda()
        a = call_noalloc(occ_d, d_max)
        b = call_workspace(occ_d, d_max)
        torch.cuda.synchronize()
        assert torch.equal(a, b), f"shape {occ.shape}, d_max {d_max}"
        outs.append(a.cpu().numpy())
    ref = oracle.edt_uncapped(small) if d_max == 0 else oracle.edt_separable(small, d_max)
    assert np.array_equal(outs[1], ref)


def test_grid_beyond_the_static_buffer_is_refused():
    nz, ny, nx = 129, 256, 256                      # one z-plane more than fits
    occ = torch.zeros((nz, ny, nx), dtype=torch.uint8, device="cuda")
    out = torch.full((nz, ny, nx), -5, dtype=torch.int32, device="cuda")
    rc = lib().edt_dense_global_noalloc(nx, ny, nz, 0, vp(occ), vp(out), stream())
    assert rc == -3                                 # EDT_ERR_CAPACITY
    torch.cuda.synchronize()
    assert bool((out == -5).all())
