"""The paper's Algorithm 1 on the CPU (oracle.Alg1) against the exact field:
it never reports less than the exact squared distance (every value comes
from a real obstacle), it is exact at obstacles and at the cap, it matches
the exact field on the boxes maps through global builds and update batches,
and on the tunnel walls it deviates in a small fraction of voxels (the
nearest-obstacle pointers travel between 26-neighbours, which is not always
enough), by a few units of squared distance."""
import numpy as np

import oracle
import workloads


def check_bounds(f, ref, occ, dmax):
    assert (f >= ref).all(), "Algorithm 1 below the exact field"
    assert (f[occ != 0] == 0).all()
    assert (f <= dmax * dmax).all()


def test_boxes_global_and_updates_match_exact():
    for seed in range(3):
        occ = workloads.dense_boxes(seed).copy()
        nz, ny, nx = occ.shape
        a = oracle.Alg1((nx, ny, nz), 20)
        a.set_map(occ)
        lowered, raised = a.transform()
        assert lowered >= int((oracle.edt_separable(occ, 20) < 400).sum()) and raised == 0
        f = a.field()
        ref = oracle.edt_separable(occ, 20)
        check_bounds(f, ref, occ, 20)
        assert np.array_equal(f, ref)
        rng = np.random.default_rng(seed)
        for _ in range(4):
            xyz = np.stack([rng.integers(0, nx, 200), rng.integers(0, ny, 200),
                            rng.integers(0, nz, 200)], 1)
            st = (rng.random(200) < 0.5).astype(np.uint8)
            for (x, y, z), v in zip(xyz, st):
                occ[z, y, x] = v
            a.apply(xyz, st)
            lowered, raised = a.transform()
            assert lowered > 0 and raised > 0
            f = a.field()
            ref = oracle.edt_separable(occ, 20)
            check_bounds(f, ref, occ, 20)
            assert (f != ref).mean() < 1e-3


def test_single_obstacle_waves():
    a = oracle.Alg1((9, 9, 9), 3)
    a.apply(np.array([[4, 4, 4]]), np.ones(1, np.uint8))
    lowered, raised = a.transform()
    z, y, x = np.meshgrid(np.arange(9), np.arange(9), np.arange(9), indexing="ij")
    d2 = (x - 4) ** 2 + (y - 4) ** 2 + (z - 4) ** 2
    assert np.array_equal(a.field(), np.minimum(d2, 9))
    assert lowered == int((d2 < 9).sum())          # every cell below the cap is lowered once
    a.apply(np.array([[4, 4, 4]]), np.zeros(1, np.uint8))
    lowered, raised = a.transform()
    assert (a.field() == 9).all() and raised >= int((d2 < 9).sum())


def test_deviation_on_tunnel_walls():
    occ = np.ascontiguousarray(workloads.tunnels(0)[:64, :128, :128])
    nz, ny, nx = occ.shape
    a = oracle.Alg1((nx, ny, nz), 32)
    a.set_map(occ)
    a.transform()
    f = a.field()
    ref = oracle.edt_separable(occ, 32)
    check_bounds(f, ref, occ, 32)
    bad = f != ref
    assert 0 < bad.sum() < 1e-3 * f.size
    assert (f - ref).max() <= 8
