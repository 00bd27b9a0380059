"""Batched transform of many dense maps: the fused persistent launch, the
launch per pass, the per-map launches and the CPU oracle agree bit for bit
on every map, for every schedule the autotuner may pick."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2105_04419_amd import FUSED, PER_MAP, PHASED, Batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available()
    oracle.build(force=False)


def small_maps(seed, n, lo, hi):
    rng = np.random.default_rng(seed)
    maps = []
    for _ in range(n):
        nx, ny, nz = (int(v) for v in rng.integers(lo, hi + 1, 3))
        occ = (rng.random((nz, ny, nx)) < rng.uniform(0.002, 0.05)).astype(np.uint8)
        occ |= workloads.room_layout(rng, nx, ny, nz, min_room=8)
        maps.append(occ)
    return maps


def check(b, maps, out, dmax, what):
    for i, (m, got) in enumerate(zip(maps, b.unpack(out))):
        ref = oracle.edt_separable(m, dmax)
        g = got.cpu().numpy()
        if not np.array_equal(g, ref):
            bad = np.argwhere(g != ref)
            raise AssertionError(f"{what}: map {i} shape {m.shape}: {len(bad)} mismatches, "
                                 f"first {bad[0]}")


@pytest.mark.parametrize("dmax", [1, 5, 8, 13, 24, 30, 33, 45, 50, 64])   # every window size M
def test_small_batch_all_modes(dmax):
    maps = small_maps(dmax, 7, 3, 70)
    b = Batch([(m.shape[2], m.shape[1], m.shape[0]) for m in maps], dmax)
    occ = b.pack(maps)
    f = b.run(occ, mode=FUSED)
    check(b, maps, f, dmax, "fused")
    p = b.run(occ, mode=PER_MAP)
    assert torch.equal(f, p)
    assert torch.equal(b.run(occ, mode=PHASED), p)


@pytest.mark.parametrize("tune", [
    {"lrun": 1, "chunk": 1, "schedule": 0, "waves_per_cu": 4, "wg_waves": 1},
    {"lrun": 3, "chunk": 7, "schedule": 0, "waves_per_cu": 16, "wg_waves": 2},
    {"lrun": 16, "chunk": 64, "schedule": 1, "waves_per_cu": 8, "wg_waves": 4},
    {"lrun": 64, "chunk": 2, "schedule": 1, "waves_per_cu": 1, "wg_waves": 1},
    {"lrun": 8, "chunk": 4, "schedule": 0, "waves_per_cu": 5, "wg_waves": 2},
    {"lrun": 4, "chunk": 1, "schedule": 1, "waves_per_cu": 16, "wg_waves": 8},
    {"lrun": 2, "chunk": 16, "schedule": 0, "waves_per_cu": 4, "wg_waves": 8},
])
def test_schedules_are_bit_identical(tune):
    maps = small_maps(11, 9, 8, 90)
    b = Batch([(m.shape[2], m.shape[1], m.shape[0]) for m in maps], 24)
    occ = b.pack(maps)
    ref = b.run(occ, mode=PER_MAP)
    check(b, maps, ref, 24, "per_map")
    assert torch.equal(b.run(occ, mode=FUSED, tune=tune), ref)
    assert torch.equal(b.run(occ, mode=PHASED, tune=tune), ref)
    assert torch.equal(b.run(occ, mode=PER_MAP, tune=tune), ref)
    # the autotuner's form: the mode inside the schedule
    assert torch.equal(b.run(occ, tune=dict(tune, mode=PHASED)), ref)


def test_rejects_bad_schedule():
    from paper_2105_04419_amd import EdtError
    b = Batch([(8, 8, 8)], 4)
    occ = b.pack([np.zeros((8, 8, 8), np.uint8)])
    for bad in ({"wg_waves": 3}, {"wg_waves": 16}, {"lrun": 0}, {"chunk": 2000},
                {"schedule": 2}, {"waves_per_cu": 65}):
        t = {"lrun": 8, "chunk": 4, "schedule": 0, "waves_per_cu": 8, "wg_waves": 4}
        t.update(bad)
        with pytest.raises(EdtError):
            b.run(occ, mode=FUSED, tune=t)
        with pytest.raises(EdtError):
            b.run(occ, mode=PHASED, tune=t)
    with pytest.raises(EdtError):
        b.run(occ, mode=3)


def test_full_batch_of_64_room_maps():
    """64 maps with sides U{32..256}, density U(1%, 30%) plus room layouts,
    d_max 24: fused == phased == per-map == oracle for every map."""
    maps = workloads.batch_maps(0)
    b = Batch([(m.shape[2], m.shape[1], m.shape[0]) for m in maps], 24)
    occ = b.pack(maps)
    f = b.run(occ, mode=FUSED)
    p = b.run(occ, mode=PER_MAP)
    assert torch.equal(f, p)
    tuned = {"lrun": 16, "chunk": 4, "schedule": 1, "waves_per_cu": 16, "wg_waves": 4}
    assert torch.equal(b.run(occ, mode=PHASED, tune=tuned), p)
    check(b, maps, f, 24, "fused 64 maps")


def test_rejects_large_radius():
    from paper_2105_04419_amd import EdtError
    with pytest.raises(EdtError):
        Batch([(8, 8, 8)], 65)


def test_degenerate_and_extreme_maps():
    """Single voxels, empty and full maps, and the longest side the batch
    accepts (4096) along each axis, in one batch."""
    rng = np.random.default_rng(3)
    maps = [np.ones((1, 1, 1), np.uint8), np.zeros((1, 1, 1), np.uint8),
            np.zeros((9, 10, 11), np.uint8), np.ones((7, 6, 5), np.uint8)]
    for axis in range(3):
        shape = [2, 3, 2]
        shape[axis] = 4096
        m = np.zeros(shape, np.uint8)
        m.reshape(-1)[rng.integers(0, m.size, 3)] = 1
        maps.append(m)
    for dmax in (1, 24, 64):
        b = Batch([(m.shape[2], m.shape[1], m.shape[0]) for m in maps], dmax)
        occ = b.pack(maps)
        f = b.run(occ, mode=FUSED)
        check(b, maps, f, dmax, f"degenerate d={dmax}")
        assert torch.equal(f, b.run(occ, mode=PER_MAP))
        assert torch.equal(f, b.run(occ, mode=PHASED))
    single = Batch([(33, 17, 5)], 24)
    m = (rng.random((5, 17, 33)) < 0.05).astype(np.uint8)
    out = single.run(single.pack([m]), mode=FUSED)
    check(single, [m], out, 24, "one map")


def test_run_length_changes_between_runs():
    # item offsets are kept for the last run length: switching back and forth
    # must rebuild them every time
    maps = small_maps(12, 7, 8, 80)
    b = Batch([(m.shape[2], m.shape[1], m.shape[0]) for m in maps], 24)
    occ = b.pack(maps)
    ref = b.run(occ, mode=PER_MAP)
    for lrun in (2, 16, 2, 8, 16):
        t = {"lrun": lrun, "chunk": 4, "schedule": 1, "waves_per_cu": 8, "wg_waves": 4}
        assert torch.equal(b.run(occ, mode=FUSED, tune=t), ref), lrun
        assert torch.equal(b.run(occ, mode=PHASED, tune=t), ref), lrun


def test_autotuner_picks_a_launch_mode_and_schedule(tmp_path, monkeypatch):
    from paper_2105_04419_amd import autotune
    monkeypatch.setenv("VDBEDT_CACHE", str(tmp_path))
    maps = small_maps(5, 6, 8, 60)
    b = Batch([(m.shape[2], m.shape[1], m.shape[0]) for m in maps], 16)
    occ = b.pack(maps)
    space = {"mode": [FUSED, PHASED], "lrun": [4, 16], "chunk": [4], "waves_per_cu": [8],
             "schedule": [0, 1], "wg_waves": [4]}
    best, results = autotune.tune(b, occ, space=space, reps=1)
    assert len(results) == 8 and best in [r[0] for r in results]
    assert best["mode"] in (FUSED, PHASED)
    ref = b.run(occ, mode=PER_MAP)
    check(b, maps, ref, 16, "per_map")
    assert torch.equal(b.run(occ, tune=best), ref)
    assert autotune.load(b) == best
