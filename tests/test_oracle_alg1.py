"""The paper's Algorithm 1 on the CPU (oracle.Alg1), in both schedules
(the paper's transform status and the conventional raise flag), against the
exact field: it never reports less than the exact squared distance (every
value comes from a real obstacle), it is exact at obstacles and at the cap,
it matches the exact field on the boxes maps through global builds and
update batches, and on the tunnel walls it deviates in a small fraction of
voxels (the nearest-obstacle pointers travel between 26-neighbours, which is
not always enough), by a few units of squared distance.  The transform
status processes fewer fronts than the conventional schedule when freed and
occupied cells lie next to each other (section IV-B)."""
import numpy as np
import pytest

import oracle
import workloads

SCHEDULES = ["transform_status", "conventional"]


def check_bounds(f, ref, occ, dmax):
    assert (f >= ref).all(), "Algorithm 1 below the exact field"
    assert (f[occ != 0] == 0).all()
    assert (f <= dmax * dmax).all()


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_boxes_global_and_updates_match_exact(schedule):
    for seed in range(3):
        occ = workloads.dense_boxes(seed).copy()
        nz, ny, nx = occ.shape
        a = oracle.Alg1((nx, ny, nz), 20, schedule)
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


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_single_obstacle_waves(schedule):
    a = oracle.Alg1((9, 9, 9), 3, schedule)
    a.apply(np.array([[4, 4, 4]]), np.ones(1, np.uint8))
    lowered, raised = a.transform()
    z, y, x = np.meshgrid(np.arange(9), np.arange(9), np.arange(9), indexing="ij")
    d2 = (x - 4) ** 2 + (y - 4) ** 2 + (z - 4) ** 2
    assert np.array_equal(a.field(), np.minimum(d2, 9))
    assert lowered == int((d2 < 9).sum())          # every cell below the cap is lowered once
    a.apply(np.array([[4, 4, 4]]), np.zeros(1, np.uint8))
    lowered, raised = a.transform()
    assert (a.field() == 9).all() and raised >= int((d2 < 9).sum())


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_deviation_on_tunnel_walls(schedule):
    occ = np.ascontiguousarray(workloads.tunnels(0)[:64, :128, :128])
    nz, ny, nx = occ.shape
    a = oracle.Alg1((nx, ny, nz), 32, schedule)
    a.set_map(occ)
    a.transform()
    f = a.field()
    ref = oracle.edt_separable(occ, 32)
    check_bounds(f, ref, occ, 32)
    bad = f != ref
    assert 0 < bad.sum() < 1e-3 * f.size
    assert (f - ref).max() <= 8


def moving_box_steps(n_steps, x0=10):
    """A 6^3 solid box moving one voxel along +x per step: its back face is
    freed and a new front face occupied, the situation the transform status
    targets (newly occupied and freed cells next to each other)."""
    steps = []
    for t in range(n_steps):
        rem = [(x0 + t, y, z) for z in range(20, 26) for y in range(20, 26)]
        add = [(x0 + t + 6, y, z) for z in range(20, 26) for y in range(20, 26)]
        steps.append((np.array(rem + add, np.int32),
                      np.array([0] * len(rem) + [1] * len(add), np.uint8)))
    return steps


@pytest.mark.parametrize("dmax", [5, 10])
def test_transform_status_saves_fronts_on_a_moving_obstacle(dmax):
    n = 48
    occ0 = np.zeros((n, n, n), np.uint8)
    occ0[20:26, 20:26, 10:16] = 1
    work = {}
    for schedule in SCHEDULES:
        occ = occ0.copy()
        a = oracle.Alg1((n, n, n), dmax, schedule)
        a.set_map(occ)
        a.transform()
        total = 0
        for xyz, st in moving_box_steps(6):
            a.apply(xyz, st)
            for (x, y, z), v in zip(xyz, st):
                occ[z, y, x] = v
            lowered, raised = a.transform()
            total += lowered + raised
            assert np.array_equal(a.field(), oracle.edt_separable(occ, dmax)), schedule
        work[schedule] = total
    assert work["transform_status"] < work["conventional"], work
