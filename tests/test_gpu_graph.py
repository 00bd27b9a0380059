"""The incremental transform and the scan integration captured in a graph
(HIP graphs through torch.cuda.CUDAGraph) and replayed on new inputs written
into the captured buffers: every replay, with eager work and synchronisation
in between, must equal the same call made eagerly, a cancelled replay
included (and the replays after it: the cancel mark is state on the device,
cleared within the call, since a captured call keeps its arguments).  The
dense context's update likewise, and a stream of several scans' updates
captured into one graph and run by one launch."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2105_04419_amd import DenseField, Field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    oracle.build(force=False)


def test_update_graph_replays_match_eager():
    occ = workloads.dense_boxes(3)
    nz, ny, nx = occ.shape
    n = 256
    rng = np.random.default_rng(12)
    g_field = Field((nx, ny, nz), 16)
    e_field = Field((nx, ny, nz), 16)
    g_field.global_(torch.from_numpy(occ).cuda())
    e_field.global_(torch.from_numpy(occ).cuda())
    xyz_buf = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
    st_buf = torch.zeros(n, dtype=torch.uint8, device="cuda")
    xyz_buf[:, 0] = 1                     # a valid no-op batch for the capture's warm-up
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g_field.update(xyz_buf, st_buf)   # warm-up on the side stream (as torch asks)
    torch.cuda.current_stream().wait_stream(s)
    e_field.update(xyz_buf, st_buf)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g_field.update(xyz_buf, st_buf)
    torch.cuda.synchronize()
    cur = occ.copy()
    cur[0, 0, 1] = 0                         # the warm-up batch cleared voxel (1, 0, 0)
    for t in range(8):
        xyz = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n), rng.integers(0, nz, n)],
                       1).astype(np.int32)
        st = (rng.random(n) < 0.5).astype(np.uint8)
        cancelled = t == 3
        if cancelled:
            xyz[7] = [nx, 0, 0]              # outside: the whole call is a no-op
        xyz_buf.copy_(torch.from_numpy(xyz))
        st_buf.copy_(torch.from_numpy(st))
        graph.replay()
        e_field.update(torch.from_numpy(xyz).cuda(), torch.from_numpy(st).cuda())
        torch.cuda.synchronize()
        if not cancelled:
            for (x, y, z), v in zip(xyz, st):
                cur[z, y, x] = v
        got = g_field.dense().cpu().numpy()
        assert np.array_equal(got, e_field.dense().cpu().numpy()), f"replay {t}"
        assert np.array_equal(got, oracle.edt_separable(cur, 16)), f"replay {t} vs oracle"
        assert g_field.error() == (-2 if cancelled else 0)
        assert e_field.error() == (-2 if cancelled else 0)


def test_scan_integration_graph_replays_match_eager():
    occ = workloads.dense_boxes(5)
    nz, ny, nx = occ.shape
    n = 1024
    rng = np.random.default_rng(4)
    g_field = Field((nx, ny, nz), 12)
    e_field = Field((nx, ny, nz), 12)
    g_field.global_(torch.from_numpy(occ).cuda())
    e_field.global_(torch.from_numpy(occ).cuda())
    o_buf = torch.tensor([32, 32, 16], dtype=torch.int32, device="cuda")
    e_buf = torch.full((n, 3), 32, dtype=torch.int32, device="cuda")
    e_buf[:, 2] = 16
    h_buf = torch.zeros(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g_field.integrate_scan(o_buf, e_buf, h_buf)
    torch.cuda.current_stream().wait_stream(s)
    e_field.integrate_scan(o_buf, e_buf, h_buf)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g_field.integrate_scan(o_buf, e_buf, h_buf)
    torch.cuda.synchronize()
    for t in range(5):
        origin = rng.integers(0, [nx, ny, nz]).astype(np.int32)
        ends = rng.integers(0, [nx, ny, nz], (n, 3)).astype(np.int32)
        hits = (rng.random(n) < 0.5).astype(np.uint8)
        o_buf.copy_(torch.from_numpy(origin))
        e_buf.copy_(torch.from_numpy(ends))
        h_buf.copy_(torch.from_numpy(hits))
        graph.replay()
        e_field.integrate_scan(torch.from_numpy(origin).cuda(), torch.from_numpy(ends).cuda(),
                               torch.from_numpy(hits).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(g_field.occupancy().cpu().numpy(), e_field.occupancy().cpu().numpy())
        assert np.array_equal(g_field.dense().cpu().numpy(), e_field.dense().cpu().numpy()), t
        assert g_field.error() == 0


def test_dense_context_graph_replays_match_eager():
    occ = workloads.dense_boxes(4)
    nz, ny, nx = occ.shape
    n = 128
    rng = np.random.default_rng(21)
    g_field = DenseField((nx, ny, nz), 0, max_changes=n)
    e_field = DenseField((nx, ny, nz), 0, max_changes=n)
    g_field.global_(torch.from_numpy(occ).cuda())
    e_field.global_(torch.from_numpy(occ).cuda())
    xyz_buf = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
    st_buf = torch.zeros(n, dtype=torch.uint8, device="cuda")
    xyz_buf[:, 0] = 1                     # a valid batch for the capture's warm-up
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g_field.update(xyz_buf, st_buf)
    torch.cuda.current_stream().wait_stream(s)
    e_field.update(xyz_buf, st_buf)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g_field.update(xyz_buf, st_buf)
    torch.cuda.synchronize()
    cur = occ.copy()
    cur[0, 0, 1] = 0
    for t in range(6):
        xyz = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n), rng.integers(0, nz, n)],
                       1).astype(np.int32)
        st = (rng.random(n) < 0.5).astype(np.uint8)
        cancelled = t in (2, 3)                  # two cancelled replays in a row, then more
        if cancelled:
            xyz[5] = [0, ny, 0]
        xyz_buf.copy_(torch.from_numpy(xyz))
        st_buf.copy_(torch.from_numpy(st))
        graph.replay()
        e_field.update(torch.from_numpy(xyz).cuda(), torch.from_numpy(st).cuda())
        torch.cuda.synchronize()
        if not cancelled:
            for (x, y, z), v in zip(xyz, st):
                cur[z, y, x] = v
        got = g_field.field().cpu().numpy()
        assert np.array_equal(got, e_field.field().cpu().numpy()), f"replay {t}"
        assert np.array_equal(got, oracle.edt_uncapped(cur)), f"replay {t} vs oracle"
        assert g_field.error() == (-2 if cancelled else 0)
        assert e_field.error() == (-2 if cancelled else 0)


def test_stream_of_updates_in_one_graph():
    # several scans' updates (each its own change list) captured together
    # and run by one graph launch equal the same updates made eagerly
    occ = workloads.dense_boxes(6)
    nz, ny, nx = occ.shape
    rng = np.random.default_rng(5)
    lists = []
    cur = occ.copy()
    for t in range(6):
        n = int(rng.integers(20, 300))
        xyz = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n), rng.integers(0, nz, n)],
                       1).astype(np.int32)
        st = (rng.random(n) < (0.6 if t % 2 == 0 else 0.3)).astype(np.uint8)
        lists.append((torch.from_numpy(xyz).cuda(), torch.from_numpy(st).cuda()))
        for (x, y, z), v in zip(xyz, st):
            cur[z, y, x] = v
    fields = [Field((nx, ny, nz), 16) for _ in range(3)]
    for f in fields:
        f.global_(torch.from_numpy(occ).cuda())
    eager, warm, g_field = fields
    for x, s in lists:
        eager.update(x, s)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        warm.update(*lists[0])
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for x, s in lists:
            g_field.update(x, s)
    torch.cuda.synchronize()
    want = oracle.edt_separable(cur, 16)
    assert np.array_equal(eager.dense().cpu().numpy(), want)
    for rep in range(2):           # the same absolute changes again end at the same map
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(g_field.dense().cpu().numpy(), want), f"launch {rep}"
        assert g_field.error() == 0
