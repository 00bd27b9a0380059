"""Autotuner for the batched transform's schedule.

The search space is the launch mode and its schedule:
  mode          FUSED (one persistent launch, grid barriers between the
                passes) or PHASED (one launch per pass)
  lrun          blocks per work item along y and z
  chunk         work items taken per queue atomic
  waves_per_cu  waves resident per compute unit (grid size of the launch)
  schedule      0 = dynamic queue, 1 = static stride
  wg_waves      waves per workgroup
Each candidate is timed with HIP events (median of `reps` runs after one
warm-up run) on the caller's batch; the winner is cached in a JSON file keyed
by GPU architecture, total-size bucket (log2 of voxels) and d_max.  Every
candidate computes the same bits (tests check this), so tuning only changes
speed.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import torch

from . import FUSED, PHASED, Batch

SPACE = {
    "mode": [FUSED, PHASED],
    "lrun": [4, 8, 16, 32],
    "chunk": [4, 16],
    "waves_per_cu": [8, 16, 32],
    "schedule": [0, 1],
    "wg_waves": [1, 4, 8],
}


def cache_path() -> str:
    d = os.environ.get("VDBEDT_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "vdbedt"))
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, "tune.json")


def arch_name() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def bucket_key(batch: Batch) -> str:
    return f"batch:{arch_name()}:v{int(math.log2(max(batch.total, 1)))}:d{batch.d_max}"


def load(batch: Batch):
    try:
        with open(cache_path()) as f:
            return json.load(f).get(bucket_key(batch))
    except (OSError, ValueError):
        return None


def store(batch: Batch, cfg: dict):
    path = cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data[bucket_key(batch)] = cfg
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_config(batch: Batch, occ, out, cfg: dict, reps: int = 5, mode: int | None = None) -> float:
    """Median milliseconds of one batched run with schedule `cfg` (launch
    mode: `mode`, else the schedule's own, else FUSED)."""
    if mode is None:
        mode = cfg.get("mode", FUSED)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    batch.run(occ, out, mode=mode, tune=cfg)
    times = []
    for _ in range(reps):
        e0.record()
        batch.run(occ, out, mode=mode, tune=cfg)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def tune(batch: Batch, occ, out=None, space: dict | None = None, reps: int = 5,
         use_cache: bool = True):
    """Search the schedule space for the fused launch.  Returns
    (best config, list of (config, ms)).  The winner is cached."""
    space = space or SPACE
    if out is None:
        out = torch.empty(batch.total, dtype=torch.int32, device=batch.device)
    results = []
    keys = list(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        cfg = dict(zip(keys, vals))
        results.append((cfg, time_config(batch, occ, out, cfg, reps)))
    best = min(results, key=lambda r: r[1])[0]
    if use_cache:
        store(batch, best)
    return best, results
