#!/usr/bin/env python
"""Benchmark of the exact truncated EDT on one MI355X.

One step = one global transform (edt_global) of the sparse tunnel map,
1024 x 1024 x 128 voxels stored as 8^3 leaf blocks (~5% of blocks hold
walls), d_max = 32, int32 output, with the block list already resident in
HBM.  `value` is extent voxels per second.  The same JSON line also reports:
  roofline       dominant kernel of the step, algorithmic bytes / its mean
                 HIP-event duration, against 8 TB/s;
  cpu_baseline   the CPU oracle (separable windowed minimum, OpenMP) on the
                 same map;
  incremental    p50 / p99 latency of edt_update over simulated range scans
                 along the tunnels, plus an incremental == global check, and
                 the same scans replayed from one captured HIP graph, and
                 the whole stream of scans back to back and as one graph;
  clearance      clearance cost forward + backward on the 64x64x32 map field
                 with 4096 x 64 waypoints, points per second;
  batched        64 dense room maps (sides 32..256, d_max 24): autotuned
                 launch (fused persistent or one launch per pass, and the
                 schedule) vs per-map launches;
  dense_small    the 64x64x32 boxes map (d_max 20), microseconds per
                 global transform;
  interior       interior distances (edt_interior) of the tunnel map's
                 occupied voxels, the inside half of the signed field;
  integrate      the same scans given as rays (sensor voxel, end voxels,
                 returns): occupancy integration on the GPU plus the
                 incremental transform, p50 / p99 per scan;
  uncapped       the full transform without a radius (int32) of the tunnel
                 map's dense extent, the paper's dataset setting, and the
                 same range scans applied to it incrementally;
  paper_alg1_cpu the paper's own Algorithm 1 on one CPU thread: a global
                 build of a tunnel-map corner (and its deviation from the
                 exact field) and range scans on the 64x64x32 map.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("voxels/s global EDT + p50/p99 incremental update latency; "
          "clearance fwd+bwd pts/s")
HBM_PEAK_GBS = 8000.0
STEP_FLOOR_B = 4.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q))


KERNEL_SOURCES = ("edt_api.hip", "edt_dev.h", "edt_kernels.hip", "edt_win.h")


def kernel_source_sha256() -> str:
    """Digest of the sources that define the global-transform kernels and
    their launches; a committed counter summary holds only for this digest."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2105_04419_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_record(kernel: str, kind: str, field: str):
    """A per-launch figure from the committed rocprofv3 counter summary
    profiles/{kernel}_tunnel_{kind}.md, or None if absent or taken on other
    kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_tunnel_{kind}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    b = re.search(field + r":\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_source_sha256():
        return None
    return float(b.group(1))


def bench_global(args, torch, np):
    """The timed steps run with nothing recorded between their kernels.  The
    per-phase split comes from a separate run with HIP events around every
    phase, and the dominant kernel's duration from a third run of as many
    steps with events around that kernel only."""
    import workloads
    from paper_2105_04419_amd import Field
    occ = workloads.tunnels(args.seed)
    nz, ny, nx = occ.shape
    bxyz, bocc = workloads.dense_to_blocks(occ)
    xyz_d = torch.from_numpy(bxyz).cuda()
    occ_d = torch.from_numpy(bocc).cuda()
    f = Field((nx, ny, nz), args.dmax)
    for _ in range(args.warmup):
        f.global_blocks(xyz_d, occ_d)
    torch.cuda.synchronize()
    st = f.stats()
    assert st["error"] == 0, st

    def timed(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            f.global_blocks(xyz_d, occ_d)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    ms = timed(args.steps)
    f.timing_begin(min(args.steps, 20))
    timed(min(args.steps, 20))
    ph = f.timing_read()
    kern = max(("pass_x", "pass_y", "pass_z"), key=lambda k: ph[k])
    f.timing_begin(args.steps, kern)
    ms_armed = timed(args.steps)
    dom_ms = f.timing_read()[kern]
    f.timing_begin(0)
    n_ext = nx * ny * nz
    n_c = st["blocks"] * 512
    return dict(f=f, occ=occ, st=st, ms=ms, phases=ph, dominant=kern, dominant_ms=dom_ms,
                ms_armed=ms_armed, n_ext=n_ext, n_c=n_c, n_obst_blocks=len(bxyz), xyz_d=xyz_d,
                occ_d=occ_d)


def roofline(g, dmax):
    """Dominant kernel of the global step and its algorithmic HBM bytes per
    launch, nb region blocks of 512 voxels:
      pass_x  reads 64 B of occupancy bits, writes a 2 B block minimum and,
              unless the block is D everywhere (then nothing reads it), 1 KiB
              of g1 (uint16); the figure counts the 1 KiB for every block, an
              upper bound;
      pass_y  reads g1 and a block minimum, writes g2 and its minimum
              (2 + 2 B per voxel, 4 B per block; an upper bound, as blocks D
              everywhere are not read, nor written in a column whose window
              is D everywhere);
      pass_z  reads g2 and its minimum, writes s (uint16) and the int32 block
              maximum (2 + 2 B per voxel, 6 B per block)."""
    nb = g["st"]["blocks"]
    per_launch = {
        "pass_x": nb * (64 + 1024 + 2),
        "pass_y": nb * (512 * 4 + 4),
        "pass_z": nb * (512 * 4 + 6),
    }
    R = (dmax + 7) // 8
    names = ({"pass_x": f"k_pass_x_rows<{R}>", "pass_y": f"k_pass_win_tiles<{R},1>",
              "pass_z": f"k_pass_win_tiles<{R},2>"} if R <= 8 else
             {"pass_x": "k_pass_x", "pass_y": "k_pass_y", "pass_z": "k_pass_z"})
    kern = g["dominant"]
    ms = g["dominant_ms"]
    achieved = per_launch[kern] / (ms * 1e-3) / 1e9
    tr = counter_record(kern, "traffic", "traffic_bytes_per_launch")
    valu = counter_record(kern, "traffic", "valu_insts_per_launch")
    return {
        "kernel": names[kern],
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": tr,
        "algorithmic_bytes_per_launch": per_launch[kern],
        "mean_ms": round(ms, 5),
        "timing": "HIP events around this kernel only, on its launch stream, over "
                  "a run of as many steps as the timed run",
        # share of the VALU issue cycles of all 1024 SIMDs at 2.4 GHz that the
        # kernel's counted VALU instructions fill (4 cycles per wave64 op)
        "valu_busy_frac": (round(valu * 4 / (1024 * 2.4e9 * ms * 1e-3), 3)
                           if valu is not None else None),
    }


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_cpu(g, args, np):
    import oracle
    oracle.build(force=False)
    nthreads = oracle.threads(args.cpu_threads) if args.cpu_threads else oracle.threads()
    occ = g["occ"]
    reps, t_total, ref = 0, 0.0, None
    while t_total < args.cpu_seconds and reps < 20:
        t0 = time.perf_counter()
        ref = oracle.edt_separable(occ, args.dmax)
        t_total += time.perf_counter() - t0
        reps += 1
    return {
        "value": g["n_ext"] * reps / t_total,
        "unit": "voxels/s",
        "cores": nthreads,
        "cpu": cpu_model(),
        "kind": "oracle",
        "sample": f"separable oracle on the full {occ.shape[2]}x{occ.shape[1]}x{occ.shape[0]} "
                  f"tunnel extent, d_max {args.dmax}, {reps} run(s), {t_total:.1f} s",
        "ms_per_map": round(t_total / reps * 1e3, 1),
    }, ref


def bench_cpu_single(g, args, np):
    """The oracle on one host thread (the paper times its method on one
    core): one full separable transform of the tunnel extent."""
    import oracle
    prev = oracle.threads()
    oracle.threads(1)
    t0 = time.perf_counter()
    oracle.edt_separable(g["occ"], args.dmax)
    t = time.perf_counter() - t0
    oracle.threads(prev)
    return {"value": g["n_ext"] / t, "unit": "voxels/s", "cores": 1, "kind": "oracle",
            "sample": f"one separable oracle run on the full tunnel extent, {t:.1f} s"}


def bench_paper_alg1(g, args, np):
    """The paper's own procedure (Algorithm 1, one CPU thread, oracle.Alg1):
    a global build of a 256 x 256 x 128 corner of the tunnel map and its
    deviation from the exact field, then 30 range scans on the 64 x 64 x 32
    boxes map (d_max 20) with per-scan time and lowered / raised fronts, the
    counts of the paper's Table II, in the paper's transform-status schedule
    and in the conventional one."""
    import oracle
    import workloads
    from workloads.scans import ScanSim, ellipse_path
    sub = np.ascontiguousarray(g["occ"][:, :256, :256])
    nz, ny, nx = sub.shape
    a = oracle.Alg1((nx, ny, nz), args.dmax)
    t0 = time.perf_counter()
    a.set_map(sub)
    lowered, _ = a.transform()
    t = time.perf_counter() - t0
    f = a.field()
    ref = oracle.edt_separable(sub, args.dmax)
    a.close()
    out = {"global": {"workload": f"tunnel map corner {nx}x{ny}x{nz}, d_max {args.dmax}",
                      "ms": round(t * 1e3, 1), "voxels_per_s": sub.size / t,
                      "lowered": lowered, "voxels_differing_from_exact": int((f != ref).sum()),
                      "max_overestimate": int((f - ref).max())}}
    occ = workloads.dense_boxes(0)
    # the paper's transform-status schedule and the conventional one on the
    # same 30 scans: per-scan time and the lowered / raised fronts (Table II)
    for schedule, key in (("transform_status", "incremental"),
                          ("conventional", "incremental_conventional")):
        sim = ScanSim(occ, ellipse_path(64, 64, 32), seed=0)
        b = oracle.Alg1((64, 64, 32), 20, schedule)
        b.set_map(occ)
        b.transform()
        ms, lo, ra, ch = [], [], [], []
        for _ in range(30):
            xyz, st, _ = sim.step()
            t0 = time.perf_counter()
            b.apply(xyz, st)
            l, r = b.transform()
            ms.append((time.perf_counter() - t0) * 1e3)
            lo.append(l)
            ra.append(r)
            ch.append(len(xyz))
        exact = bool(np.array_equal(b.field(), oracle.edt_separable(sim.map, 20)))
        b.close()
        out[key] = {"workload": "30 range scans on the 64x64x32 boxes map, d_max 20",
                    "schedule": schedule,
                    "p50_ms": round(pct(ms, 50), 3), "changed_mean": float(np.mean(ch)),
                    "lowered_mean": float(np.mean(lo)), "raised_mean": float(np.mean(ra)),
                    "equals_exact": exact}
    out["cores"] = 1
    return out


def bench_tunnel_x4(args, torch, np):
    """The tunnel map tiled 2 x 2 in x and y (2048 x 2048 x 128 extent, four
    times the region): its pool and intermediates exceed the 256 MB last-level
    cache, so the pass rates here are HBM rates."""
    import workloads
    from paper_2105_04419_amd import Field
    occ = workloads.tunnels(args.seed)
    nz, ny, nx = occ.shape
    bxyz, bocc = workloads.dense_to_blocks(occ)
    tiles = []
    for j in range(2):
        for i in range(2):
            t = bxyz.copy()
            t[:, 0] += i * (nx // 8)
            t[:, 1] += j * (ny // 8)
            tiles.append(t)
    xyz_d = torch.from_numpy(np.concatenate(tiles)).cuda()
    occ_d = torch.from_numpy(np.concatenate([bocc] * 4)).cuda()
    f = Field((2 * nx, 2 * ny, nz), args.dmax)
    for _ in range(2):
        f.global_blocks(xyz_d, occ_d)
    torch.cuda.synchronize()
    steps = max(3, args.steps // 2)
    f.timing_begin(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f.global_blocks(xyz_d, occ_d)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ph = f.timing_read()
    f.timing_begin(0)
    st = f.stats()
    assert st["error"] == 0, st
    nb = st["blocks"]
    per_voxel = {"pass_x": (64 + 1024 + 2) / 512, "pass_y": 4 + 4 / 512, "pass_z": 4 + 6 / 512}
    return {
        "workload": f"tunnel map tiled 2x2: {2 * nx}x{2 * ny}x{nz}, d_max {args.dmax}",
        "region_blocks": nb,
        "ms_per_transform": round(ms, 4),
        "extent_voxels_per_s": 4 * nx * ny * nz / (ms * 1e-3),
        "region_voxels_per_s": nb * 512 / (ms * 1e-3),
        "phases_ms": {k: round(v, 5) for k, v in ph.items() if k != "calls"},
        "pass_algorithmic_GBps": {k: round(nb * 512 * v / (ph[k] * 1e-3) / 1e9, 1)
                                  for k, v in per_voxel.items()},
    }


def scan_lists(g, args, np):
    """The change lists of the simulated range scans along the tunnels (and
    the map after the last scan), generated once and cached."""
    import workloads
    from workloads.scans import ScanSim, tunnel_path
    cache = os.path.join(workloads.cache_dir(), f"scans_tunnel_s{args.seed}_{args.scans}.npz")
    if os.path.exists(cache):
        z = np.load(cache)
        lists = [(z[f"x{i}"], z[f"s{i}"]) for i in range(args.scans)]
        final = z["final"]
    else:
        sim = ScanSim(g["occ"], tunnel_path(args.seed), seed=args.seed)
        lists = []
        for _ in range(args.scans):
            x, s, _ = sim.step()
            lists.append((x, s))
        final = sim.map
        np.savez(cache + ".tmp.npz", final=final,
                 **{f"x{i}": x for i, (x, _) in enumerate(lists)},
                 **{f"s{i}": s for i, (_, s) in enumerate(lists)})
        os.replace(cache + ".tmp.npz", cache)
    return lists, final


def bench_incremental(g, args, torch, np):
    from paper_2105_04419_amd import Field
    lists, final = scan_lists(g, args, np)
    f = g["f"]
    f.global_blocks(g["xyz_d"], g["occ_d"])
    dev = [(torch.from_numpy(x).cuda(), torch.from_numpy(s).cuda()) for x, s in lists]
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    dev_ms, wall_ms, changed, dirty = [], [], [], []
    for i, (x, s) in enumerate(dev):
        t0 = time.perf_counter()
        e0.record()
        f.update(x, s)
        e1.record()
        e1.synchronize()
        t1 = time.perf_counter()
        if i >= args.scan_warmup:
            dev_ms.append(e0.elapsed_time(e1))
            wall_ms.append((t1 - t0) * 1e3)
            st = f.stats()
            changed.append(st["changed"])
            dirty.append(st["dirty_blocks"])
    h = Field(f.shape, args.dmax)
    h.global_(torch.from_numpy(final).cuda())
    same = bool(torch.equal(h.dense(), f.dense()))
    graph = bench_incremental_graph(g, args, torch, np, dev, h)
    stream = bench_incremental_stream(g, args, torch, np, dev, h)
    return {
        "scans": len(dev_ms),
        "p50_ms": round(pct(dev_ms, 50), 4),
        "p99_ms": round(pct(dev_ms, 99), 4),
        "host_p50_ms": round(pct(wall_ms, 50), 4),
        "host_p99_ms": round(pct(wall_ms, 99), 4),
        "changed_voxels_mean": round(float(np.mean(changed)), 1),
        "dirty_blocks_mean": round(float(np.mean(dirty)), 1),
        "incremental_equals_global": same,
        "graph": graph,
        "stream": stream,
    }


def bench_incremental_stream(g, args, torch, np, dev, final_field):
    """The scans as one stream of updates: enqueued back to back with no
    synchronisation between them, and captured together into one HIP graph
    (every scan's own change list, unpadded) that one launch runs.  Device
    time per scan over the whole stream; the field after it against the
    global transform of the final map."""
    from paper_2105_04419_amd import Field
    todo = [(x, s) for x, s in dev if x.shape[0] > 0]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # back to back, eager
    f = Field(g["f"].shape, args.dmax)
    f.global_blocks(g["xyz_d"], g["occ_d"])
    torch.cuda.synchronize()
    e0.record()
    for x, s in todo:
        f.update(x, s)
    e1.record()
    e1.synchronize()
    eager_ms = e0.elapsed_time(e1)
    eager_same = bool(torch.equal(final_field.dense(), f.dense())) and f.error() == 0
    # one graph of all the scans' updates; warm-up on another field
    w = Field(g["f"].shape, args.dmax)
    w.global_blocks(g["xyz_d"], g["occ_d"])
    q = Field(g["f"].shape, args.dmax)
    q.global_blocks(g["xyz_d"], g["occ_d"])
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        w.update(*todo[0])
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for x, s in todo:
            q.update(x, s)
    torch.cuda.synchronize()
    # the first launch uploads the graph; the second runs the same absolute
    # changes again from the final map, which ends at the same map
    times = []
    for _ in range(2):
        e0.record()
        graph.replay()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    graph_same = bool(torch.equal(final_field.dense(), q.dense())) and q.error() == 0
    del graph
    return {
        "scans": len(todo),
        "eager_back_to_back_ms_per_scan": round(eager_ms / len(todo), 4),
        "one_graph_ms_per_scan": round(times[-1] / len(todo), 4),
        "one_graph_first_launch_ms_per_scan": round(times[0] / len(todo), 4),
        "kernels_per_scan": 6,
        "stream_equals_global": eager_same and graph_same,
    }


def bench_incremental_graph(g, args, torch, np, dev, final_field):
    """The same scans replayed from one captured HIP graph of edt_update: the
    change lists are padded to the longest (repeating the last entry, a
    no-op) and copied into the captured buffers before each replay; a scan
    without changes needs no update and is not replayed."""
    from paper_2105_04419_amd import Field
    n = max(int(x.shape[0]) for x, _ in dev)
    pad = []
    for x, s in dev:
        k = n - x.shape[0]
        if x.shape[0] == 0:
            pad.append(None)
            continue
        pad.append((torch.cat([x, x[-1:].expand(k, 3)]) if k else x,
                    torch.cat([s, s[-1:].expand(k)]) if k else s))
    first = next(p for p in pad if p is not None)
    f = Field(g["f"].shape, args.dmax)
    f.global_blocks(g["xyz_d"], g["occ_d"])
    xb = torch.empty((n, 3), dtype=torch.int32, device="cuda")
    sb = torch.empty(n, dtype=torch.uint8, device="cuda")
    # capture on a copy of the first scan, after a warm-up of the same call
    w = Field(g["f"].shape, args.dmax)
    w.global_blocks(g["xyz_d"], g["occ_d"])
    xb.copy_(first[0])
    sb.copy_(first[1])
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        w.update(xb, sb)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        f.update(xb, sb)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    dev_ms, wall_ms = [], []
    for i, p in enumerate(pad):
        if p is None:
            continue
        xb.copy_(p[0])
        sb.copy_(p[1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        graph.replay()
        e1.record()
        e1.synchronize()
        t1 = time.perf_counter()
        if i >= args.scan_warmup:
            dev_ms.append(e0.elapsed_time(e1))
            wall_ms.append((t1 - t0) * 1e3)
    assert f.error() == 0
    return {
        "padded_changes": n,
        "p50_ms": round(pct(dev_ms, 50), 4),
        "p99_ms": round(pct(dev_ms, 99), 4),
        "host_p50_ms": round(pct(wall_ms, 50), 4),
        "host_p99_ms": round(pct(wall_ms, 99), 4),
        "graph_equals_global": bool(torch.equal(final_field.dense(), f.dense())),
    }


def bench_integrate(g, args, torch, np):
    """Occupancy integration of the scans' rays on the GPU followed by the
    incremental transform (edt_integrate_scan), per scan."""
    import workloads
    from workloads.scans import ScanSim, tunnel_path
    from paper_2105_04419_amd import Field
    n_scans = args.scans
    cache = os.path.join(workloads.cache_dir(), f"rays_tunnel_s{args.seed}_{n_scans}.npz")
    if os.path.exists(cache):
        z = np.load(cache)
        scans = [(z[f"p{i}"], z[f"e{i}"], z[f"h{i}"]) for i in range(n_scans)]
    else:
        sim = ScanSim(g["occ"], tunnel_path(args.seed), seed=args.seed)
        scans = [sim.rays() for _ in range(n_scans)]
        np.savez(cache + ".tmp.npz", **{f"p{i}": p for i, (p, _, _) in enumerate(scans)},
                 **{f"e{i}": e for i, (_, e, _) in enumerate(scans)},
                 **{f"h{i}": h for i, (_, _, h) in enumerate(scans)})
        os.replace(cache + ".tmp.npz", cache)
    nz, ny, nx = g["occ"].shape
    f = Field((nx, ny, nz), args.dmax)
    f.global_blocks(g["xyz_d"], g["occ_d"])
    dev = [tuple(torch.from_numpy(a).cuda() for a in sc) for sc in scans]
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    dev_ms, changed = [], []
    for i, (p, e, h) in enumerate(dev):
        e0.record()
        f.integrate_scan(p, e, h)
        e1.record()
        e1.synchronize()
        if i >= args.scan_warmup:
            dev_ms.append(e0.elapsed_time(e1))
            changed.append(f.stats()["changed"])
    assert f.error() == 0
    h2 = Field(f.shape, args.dmax)
    h2.global_(f.occupancy())
    same = bool(torch.equal(h2.dense(), f.dense()))
    return {
        "workload": f"tunnel map, {len(scans[0][1])} rays per scan (16 x 1024, range 150), "
                    f"d_max {args.dmax}",
        "scans": len(dev_ms),
        "p50_ms": round(pct(dev_ms, 50), 4),
        "p99_ms": round(pct(dev_ms, 99), 4),
        "changed_voxels_mean": round(float(np.mean(changed)), 1),
        "integrated_equals_global": same,
    }


def bench_readback(g, args, torch, np):
    """Dense readbacks of the tunnel map (edt_read_dense: int32 field of the
    whole extent; edt_read_occupancy: uint8).  Algorithmic bytes: the output,
    plus the stored uint16 field (64 B of bits for the occupancy) of every
    region block."""
    f = g["f"]
    f.global_blocks(g["xyz_d"], g["occ_d"])
    nz, ny, nx = g["occ"].shape
    out = torch.empty((nz, ny, nx), dtype=torch.int32, device="cuda")
    occo = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
    nb = g["st"]["blocks"]
    res = {}
    for name, fn, nbytes in (("field_int32", lambda: f.dense(out=out), 4 * g["n_ext"] + 1024 * nb),
                             ("occupancy_u8", lambda: f.occupancy(out=occo), g["n_ext"] + 64 * nb)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        n = 20
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / n
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"ms": round(ms, 4), "algorithmic_bytes": nbytes, "GB_per_s": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    # None when the CPU oracle did not run (--no-cpu)
    res["field_equals_oracle"] = (None if g.get("parity_ref") is None else
                                  bool(np.array_equal(out.cpu().numpy(), g["parity_ref"])))
    return res


def bench_clearance(args, torch, np):
    import workloads
    from paper_2105_04419_amd import ClearanceCost, Field
    occ = workloads.dense_boxes(0)
    f = Field((64, 64, 32), 20)
    f.global_(torch.from_numpy(occ).cuda())
    s = f.dense()
    wp = torch.from_numpy(workloads.trajectories(0, occ)).cuda()
    n = wp.shape[0] * wp.shape[1]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    times = []
    for r in range(args.clear_reps + 5):
        x = wp.detach().requires_grad_(True)
        e0.record()
        c = ClearanceCost.apply(s, x, 0.2, 1.0)
        c.sum().backward()
        e1.record()
        e1.synchronize()
        if r >= 5:
            times.append(e0.elapsed_time(e1))
    med = pct(times, 50)
    # the two kernels alone, without autograd's dispatch between them
    from paper_2105_04419_amd import clearance_bwd, clearance_fwd
    gc = torch.ones(wp.shape[0], device="cuda")
    cost = torch.empty(wp.shape[0], dtype=torch.float32, device="cuda")
    gwp = torch.empty_like(wp)
    dev = []
    for r in range(args.clear_reps + 5):
        e0.record()
        clearance_fwd(s, wp, 0.2, 1.0, out=cost)
        clearance_bwd(s, wp, gc, 0.2, 1.0, out=gwp)
        e1.record()
        e1.synchronize()
        if r >= 5:
            dev.append(e0.elapsed_time(e1))
    dmed = pct(dev, 50)
    return {"points": n, "median_ms": round(med, 4), "pts_per_s": n / (med * 1e-3),
            "timing": "HIP events around forward + backward through torch.autograd",
            "kernels_median_ms": round(dmed, 4), "kernels_pts_per_s": n / (dmed * 1e-3)}


def bench_batch(args, torch, np):
    import workloads
    from paper_2105_04419_amd import FUSED, PER_MAP, PHASED, DEFAULT_TUNE, Batch, autotune
    maps = workloads.batch_maps(args.seed)
    b = Batch([(m.shape[2], m.shape[1], m.shape[0]) for m in maps], 24)
    occ = b.pack(maps)
    out = torch.empty(b.total, dtype=torch.int32, device=b.device)
    best, results = autotune.tune(b, occ, out, reps=3)
    best_of = {m: min((r for r in results if r[0]["mode"] == m), key=lambda r: r[1])[0]
               for m in (FUSED, PHASED)}
    reps = 10
    t_tuned = autotune.time_config(b, occ, out, best, reps)
    t_mode = {m: autotune.time_config(b, occ, out, c, reps) for m, c in best_of.items()}
    t_default = autotune.time_config(b, occ, out, DEFAULT_TUNE, reps, mode=FUSED)
    per_map_cfg = dict(DEFAULT_TUNE, lrun=best["lrun"])
    t_per_map = autotune.time_config(b, occ, out, per_map_cfg, reps, mode=PER_MAP)
    tuned = b.run(occ, tune=best).clone()
    per_map = b.run(occ, mode=PER_MAP, tune=per_map_cfg)
    fused = b.run(occ, tune=best_of[FUSED])
    nvox = b.total
    names = {FUSED: "fused", PHASED: "phased"}
    return {
        "maps": len(maps),
        "voxels": nvox,
        "d_max": 24,
        "tuned_ms": round(t_tuned, 4),
        "tuned_voxels_per_s": nvox / (t_tuned * 1e-3),
        "tuned_schedule": dict(best, mode=names[best["mode"]]),
        "fused_ms": round(t_mode[FUSED], 4),
        "phased_ms": round(t_mode[PHASED], 4),
        "fused_default_schedule_ms": round(t_default, 4),
        "per_map_ms": round(t_per_map, 4),
        "per_map_voxels_per_s": nvox / (t_per_map * 1e-3),
        "speedup_tuned_vs_per_map": round(t_per_map / t_tuned, 3),
        "search_space": {k: ([names[m] for m in v] if k == "mode" else v)
                         for k, v in autotune.SPACE.items()},
        "trials": len(results),
        "tuned_equals_per_map": bool(torch.equal(tuned, per_map)),
        "fused_equals_per_map": bool(torch.equal(fused, per_map)),
        # floor: 1 B of occupancy read and 4 B of int32 written per voxel
        "hbm_frac_floor": round(5 * nvox / (t_tuned * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
    }


def bench_dense_small(args, torch, np):
    import workloads
    from paper_2105_04419_amd import Field
    occ = torch.from_numpy(workloads.dense_boxes(0)).cuda()
    f = Field((64, 64, 32), 20)
    for _ in range(5):
        f.global_(occ)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n = 50
    e0.record()
    for _ in range(n):
        f.global_(occ)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / n
    return {"workload": "dense 64x64x32 boxes map, d_max 20", "us_per_transform": round(ms * 1e3, 2),
            "voxels_per_s": 64 * 64 * 32 / (ms * 1e-3)}


def bench_interior(g, args, torch, np):
    """Interior distances (edt_interior) of the tunnel map's occupied voxels."""
    from paper_2105_04419_amd import Field
    nz, ny, nx = g["occ"].shape
    f = Field((nx, ny, nz), args.dmax, max_interior_blocks=g["n_obst_blocks"])
    f.global_blocks(g["xyz_d"], g["occ_d"])
    for _ in range(5):
        f.interior()
    torch.cuda.synchronize()
    assert f.error() == 0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n = 50
    e0.record()
    for _ in range(n):
        f.interior()
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / n
    nb = g["n_obst_blocks"]
    return {"workload": f"tunnel map, {nb} blocks holding an obstacle, d_max {args.dmax}",
            "ms": round(ms, 5), "block_voxels_per_s": nb * 512 / (ms * 1e-3)}


def bench_uncapped(g, args, torch, np):
    """Full transform without a radius (edt_dense_global) of the tunnel
    map's whole extent, as the paper runs its dataset benchmarks."""
    from paper_2105_04419_amd import dense_global, lib
    occ = torch.from_numpy(g["occ"]).cuda()
    nz, ny, nx = g["occ"].shape
    ws = torch.empty(int(lib().edt_dense_workspace_bytes(nx, ny, nz)), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty((nz, ny, nx), dtype=torch.int32, device="cuda")
    for _ in range(3):
        dense_global(occ, 0, out, ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n = 10
    e0.record()
    for _ in range(n):
        dense_global(occ, 0, out, ws)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / n
    vox = nx * ny * nz
    res = {"workload": f"tunnel map {nx}x{ny}x{nz}, dense input, no radius, int32 output",
           "ms": round(ms, 4), "voxels_per_s": vox / (ms * 1e-3),
           "max_squared_distance": int(out.max().item())}
    del ws, out
    res["incremental"] = bench_uncapped_incremental(g, args, torch, np)
    return res


def bench_uncapped_incremental(g, args, torch, np):
    """The range scans applied to the uncapped field of the whole extent
    (edt_dense_ctx_update): p50 / p99 device latency per scan, and the field
    after the last scan against the global transform of the final map."""
    from paper_2105_04419_amd import DenseField, dense_global
    lists, final = scan_lists(g, args, np)
    nz, ny, nx = g["occ"].shape
    f = DenseField((nx, ny, nz), 0, max_changes=max(1, max(len(x) for x, _ in lists)))
    f.global_(torch.from_numpy(g["occ"]).cuda())
    dev = [(torch.from_numpy(x).cuda(), torch.from_numpy(s).cuda()) for x, s in lists]
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ms = []
    for i, (x, s) in enumerate(dev):
        e0.record()
        f.update(x, s)
        e1.record()
        e1.synchronize()
        if i >= args.scan_warmup:
            ms.append(e0.elapsed_time(e1))
    same = bool(torch.equal(f.field(), dense_global(torch.from_numpy(final).cuda())))
    return {"scans": len(ms), "p50_ms": round(pct(ms, 50), 4), "p99_ms": round(pct(ms, 99), 4),
            "incremental_equals_global": same, "error": f.error()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--dmax", type=int, default=32)
    ap.add_argument("--scans", type=int, default=200)
    ap.add_argument("--scan-warmup", type=int, default=5)
    ap.add_argument("--clear-reps", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(sharding is a design, not code)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    log(f"[bench] global transform, tunnel map seed {args.seed}, d_max {args.dmax}")
    g = bench_global(args, torch, np)
    rl = roofline(g, args.dmax)
    out = {
        "metric": METRIC,
        "value": g["n_ext"] / (g["ms"] * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {
            "workload": "sparse tunnel map 1024x1024x128, 12 tubes, 8^3 leaf blocks, "
                        f"d_max {args.dmax}, int32 squared distances, seed {args.seed}",
            "obstacle_blocks": g["n_obst_blocks"],
            "region_blocks": g["st"]["blocks"],
            "region_voxels": g["n_c"],
            "extent_voxels": g["n_ext"],
            "voxels_counted": "the whole extent: the field covers every voxel, the blocks "
                              "outside the computed region hold D implicitly",
        },
        "region_voxels_per_s": g["n_c"] / (g["ms"] * 1e-3),
        # the step against a floor of 4.3 B per region voxel (an int32 field
        # write plus occupancy and block metadata), as if the step wrote int32
        "step_floor_frac": round(STEP_FLOOR_B * g["n_c"] / (g["ms"] * 1e-3) /
                                 (HBM_PEAK_GBS * 1e9), 4),
        "step_floor_bytes_per_region_voxel": STEP_FLOOR_B,
        "phases_ms": {k: round(v, 5) for k, v in g["phases"].items() if k != "calls"},
        "phases_timing": "separate run with HIP events around every phase",
        "ms_per_step_dominant_kernel_bracketed": round(g["ms_armed"], 5),
        "roofline": rl,
    }
    if not args.no_cpu:
        log("[bench] cpu oracle baseline")
        cb, ref = bench_cpu(g, args, np)
        out["cpu_baseline"] = cb
        got = g["f"].dense().cpu().numpy()
        out["parity_global_vs_oracle"] = bool(np.array_equal(got, ref))
        g["parity_ref"] = ref
        if not args.no_extra:
            log("[bench] cpu oracle, one thread")
            out["cpu_single_thread"] = bench_cpu_single(g, args, np)
            log("[bench] the paper's Algorithm 1 on one cpu thread")
            out["paper_alg1_cpu"] = bench_paper_alg1(g, args, np)
    if not args.no_extra:
        log("[bench] dense readbacks of the tunnel map")
        out["readback"] = bench_readback(g, args, torch, np)
        log(f"[bench] incremental: {args.scans} scans")
        out["incremental"] = bench_incremental(g, args, torch, np)
        log(f"[bench] scan integration + incremental: {args.scans} scans")
        out["integrate"] = bench_integrate(g, args, torch, np)
        log("[bench] clearance 4096 x 64")
        out["clearance"] = bench_clearance(args, torch, np)
        log("[bench] batched: 64 dense maps, autotuned launch vs per-map launches")
        out["batched"] = bench_batch(args, torch, np)
        log("[bench] dense 64x64x32 global transform")
        out["dense_small"] = bench_dense_small(args, torch, np)
        log("[bench] interior distances of the tunnel map")
        out["interior"] = bench_interior(g, args, torch, np)
        log("[bench] uncapped dense transform of the tunnel extent")
        out["uncapped"] = bench_uncapped(g, args, torch, np)
        log("[bench] tunnel map tiled 2x2 (working set beyond the last-level cache)")
        out["tunnel_x4"] = bench_tunnel_x4(args, torch, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
