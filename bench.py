#!/usr/bin/env python3
"""Throughput of the whole hot path -- bin, sub-sample, mesh, normals, labels --
on one MI355X, for a batch of uneven synthetic sweeps resident in HBM.

One step = the full path over the batch (64 street sweeps; rings drawn from
{16,32,64,128}, azimuth widths from {1024,2048,4096}; range noise 1 cm; 10%
dropouts; per-frame seeds), as one library call.  The batch is timed in every
launch form: the batched chain replayed from a captured hipGraph, launched
directly, launched directly with two batches in flight (two contexts and
streams taken in turn, each call still a whole pass over the batch), and as
plain per-frame chains.  `value` is points/s of the fastest form that serves
whole batches (`config.launch` names it).  The dominant kernel is timed with
HIP events for the roofline figure.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points/s mesh+normals+labels, batched-served vs plain; p50/p99 frame latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernels' code: comments and blank space left out, so that an
    edit of a comment does not invalidate counters taken on the same code."""
    import re
    h = hashlib.sha256()
    for name in ("lidarseg_kernels.hip", "lidarseg_internal.h"):
        with open(os.path.join(ROOT, "paper_2005_02704_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


STAGE_KERNEL = {"bin": "k_bin", "count": "k_count", "geom": "k_geom", "cc": "k_cc", "merge": "k_merge",
                "compress": "k_compress", "flatten": "k_flatten", "scan": "k_scan", "label": "k_resolve",
                "post": "k_post", "score": "k_score"}


def stage_bytes(stage, N, V, T):
    """Algorithmic bytes a stage must move (what the method reads and writes,
    not the key grid or other scratch).  N input points, V vertices, T triangles."""
    if stage == "bin":
        return 12 * N                         # xyz of every input point
    if stage == "geom":
        return 12 * V + 12 * V + 12 * V + 4 * V + 12 * T  # kept xyz in; vertices, normals,
        # vertex_point, triangles out
    if stage == "label":
        return 4 * V                          # labels written
    return 0


def link_rates(torch):
    """Pinned host <-> device copy rates (GB/s) of the PCIe link: 8 copies of
    64 MiB host to device, device to host, and both at once on three streams."""
    dev = torch.device("cuda", 0)
    chunk, count = 64 << 20, 8
    host = [torch.empty(chunk, dtype=torch.uint8).pin_memory() for _ in range(2 * count)]
    devm = [torch.empty(chunk, dtype=torch.uint8, device=dev) for _ in range(2 * count)]
    streams = [torch.cuda.Stream(dev) for _ in range(3)]
    out = {}
    for name, pairs in (("h2d", [(devm[i], host[i]) for i in range(count)]),
                        ("d2h", [(host[i], devm[i]) for i in range(count)]),
                        ("both", [(devm[i], host[i]) for i in range(count)] +
                                 [(host[count + i], devm[count + i]) for i in range(count)])):
        def go():
            for j, (dst, src) in enumerate(pairs):
                with torch.cuda.stream(streams[j % 3]):
                    dst.copy_(src, non_blocking=True)
            torch.cuda.synchronize()
        go()
        t = time.perf_counter()
        for _ in range(4):
            go()
        out[name + "_GB_s"] = round(chunk * len(pairs) * 4 / (time.perf_counter() - t) / 1e9, 1)
    return out


def served_run(args, lp, synth, torch):
    """8 simulated sensors (rings 16/32/64/128, widths 1024/2048/4096, 10-20 Hz
    Poisson arrivals) through the native continuous-batching server, driven by
    its native replay (no Python between arrival and completion); then the
    same sensors at a hundred times their rates for 3 s (groups form under load); then the
    pool with every request arriving at once (capacity), and for comparison the
    same burst served one sweep per call with plain per-frame launches.
    Latency runs from submission to the results in pinned host memory; every
    rate includes the points' host-to-device copies and the results' copies back,
    and the PCIe link's own copy rates bound the capacity."""
    import numpy as np
    from paper_2005_02704_amd.lidarserve import LIDAR_SERVED_OK, NativeServer
    from paper_2005_02704_amd.serve import poisson_schedule
    sensors = synth.served_sensors(8)
    n_pool = 3
    log(f"served: generating {8 * n_pool} pool sweeps")
    pool = [[synth.make_frame(s, "street", synth.frame_seed(9000 + q, k), sigma=0.01, dropout=0.10)
             for k in range(n_pool)] for q, (s, _) in enumerate(sensors)]
    geos = [lp.SensorGeometry(s.elevations(), s.n_azimuth, 1, 1, s.az0) for s, _ in sensors]
    pinned = [[torch.from_numpy(f.xyz).pin_memory() for f in row] for row in pool]
    budget = 1 << 30
    n_slots, max_batch = 4, 24

    def replay(srv, sched):
        lat, st, gs, wall = srv.replay([t for t, _, _ in sched], [q for _, q, _ in sched],
                                       [pinned[q][k] for _, q, k in sched])
        ok = st == LIDAR_SERVED_OK
        pts = sum(int(pinned[q][k].shape[0]) for (_, q, k), good in zip(sched, ok) if good)
        lat_ms = lat[ok] * 1e3
        return {"requests": int(ok.sum()), "failed": int((~ok).sum()), "points": pts,
                "points_per_s": round(pts / wall, 1),
                "p50_ms": round(float(np.percentile(lat_ms, 50)), 4) if ok.any() else None,
                "p99_ms": round(float(np.percentile(lat_ms, 99)), 4) if ok.any() else None,
                "max_ms": round(float(lat_ms.max()), 4) if ok.any() else None,
                "mean_batch": round(float(gs[ok].mean()), 3) if ok.any() else None,
                "wall_s": round(wall, 3)}

    rates = [r for _, r in sensors]
    srv = NativeServer(geos, n_slots=n_slots, max_batch=max_batch, launch=args.served_launch, sets_per_sensor=24,
                       budget_bytes=budget, timeout_s=1.0)
    burst = [(0.0, q % 8, (q // 8) % n_pool) for q in range(8 * 64)]
    replay(srv, burst)   # untimed: first touches of every set and slot
    sched = poisson_schedule(rates, args.served_seconds, seed=args.seed, n_payloads=n_pool)
    log(f"served: {len(sched)} sweeps over {args.served_seconds:.0f}s (native server, {args.served_launch})")
    stream_st = replay(srv, sched)
    log(f"  p50 {stream_st['p50_ms']:.3f} ms  p99 {stream_st['p99_ms']:.3f} ms  "
        f"{stream_st['points_per_s']:.3e} points/s  mean group {stream_st['mean_batch']}")
    heavy = poisson_schedule([100 * r for r in rates], 3.0, seed=args.seed + 1, n_payloads=n_pool)
    heavy_st = replay(srv, heavy)
    log(f"  100x rates: p50 {heavy_st['p50_ms']:.3f} ms  p99 {heavy_st['p99_ms']:.3f} ms  "
        f"{heavy_st['points_per_s']:.3e} points/s  mean group {heavy_st['mean_batch']}")
    cap_st = replay(srv, burst)
    log(f"  capacity: {cap_st['points_per_s']:.3e} points/s ({len(burst)} sweeps at once, "
        f"mean group {cap_st['mean_batch']})")
    stats = srv.stats()
    srv.close()
    # bytes the burst moves over the link: points in, each sweep's result block
    # (8 + 2 x lattice cells int32) out
    link_bytes = sum(12 * int(pinned[q][k].shape[0]) + 4 * (8 + 2 * geos[q].n_rings * geos[q].n_azimuth)
                     for _, q, k in burst)
    link = link_rates(torch)
    link["burst_bytes_per_point"] = round(link_bytes / cap_st["points"], 2)
    link["bound_points_per_s"] = round(link["both_GB_s"] * 1e9 / link["burst_bytes_per_point"], 1)
    log(f"  PCIe link: {link}")
    srv_p = NativeServer(geos, n_slots=n_slots, max_batch=1, launch="plain", sets_per_sensor=24, budget_bytes=budget,
                         timeout_s=1.0)
    replay(srv_p, burst)
    plain_st = replay(srv_p, burst)
    log(f"  capacity, one sweep per plain call: {plain_st['points_per_s']:.3e} points/s")
    srv_p.close()
    return {"workload": "8 sensors, rings 16/32/64/128, azimuth 1024/2048/4096, 10-20 Hz Poisson, "
                        f"{args.served_seconds:.0f}s, budget {budget >> 30} GiB, {n_slots} slots, groups of up to {max_batch}, "
                        f"{args.served_launch} launches, 1 s watchdog per group; native server and replay",
            **stream_st,
            "latency": "submission to labels/vertex_point/counts in pinned host memory",
            "heavy_100x_rates_3s": heavy_st,
            "capacity_points_per_s": cap_st["points_per_s"],
            "capacity_mean_batch": cap_st["mean_batch"],
            "capacity_plain_one_sweep_per_call_points_per_s": plain_st["points_per_s"],
            "pcie_link": link,
            "max_slots_in_flight": stats["max_slots_busy"], "peak_admitted_bytes": stats["peak_bytes"],
            "server_device_bytes": stats["device_bytes"]}, [f for row in pool for f in row]


def mean_scores(outs, lp):
    prf = [lp.precision_recall_f1(tuple(int(x) for x in o.edge_counts.cpu())) for o in outs]
    return {k: round(float(sum(v[j] for v in prf) / len(prf)), 4) for j, k in enumerate(("precision", "recall", "f1"))}


def accuracy_run(args, lp, synth, torch, ctx, frames, geos, stream):
    """Edge scores (segment edges against the generator's surface ids, each
    dilated by one lattice step), averaged over frames: on the benchmark batch
    (with the time of the scoring stage), and at the paper's own sweep shape
    (32 rings x 1800 firings) for sampling intervals 5, 10 and 15."""
    import numpy as np
    dev = torch.device("cuda", 0)
    params = lp.make_params(1.0, 60.0, (0.2, 0.2, 0.2), score_radius=1)
    inputs = [(torch.from_numpy(f.xyz).to(dev), g, None, torch.from_numpy(f.prim.astype(np.int32)).to(dev))
              for f, g in zip(frames, geos)]
    outs = [lp.Outputs(g, dev, scores=True) for g in geos]
    prep = ctx.prepare(inputs, params, outs)
    for _ in range(3):
        ctx.lidar_mesh_segment(prep, stream, "batched")
    torch.cuda.synchronize()
    ctx.stage_times()
    ctx.set_profiling(True)
    for _ in range(10):
        ctx.lidar_mesh_segment(prep, stream, "batched")
    torch.cuda.synchronize()
    st = ctx.stage_times()
    ctx.set_profiling(False)
    batch = {**mean_scores(outs, lp), "score_ms": round(st["score"][0] / max(st["score"][1], 1), 5)}
    log(f"  batch edge scores {batch}")
    w = synth.WORKLOADS["paper_32x1800"]
    n_env = 8
    envs = synth.workload_frames("paper_32x1800", n_env)
    paper = {}
    for s in w["s"]:
        g = [lp.SensorGeometry(f.sensor.elevations(), f.sensor.n_azimuth, s, 1, f.sensor.az0) for f in envs]
        inp = [(torch.from_numpy(f.xyz).to(dev), gg, None, torch.from_numpy(f.prim.astype(np.int32)).to(dev))
               for f, gg in zip(envs, g)]
        o = [lp.Outputs(gg, dev, scores=True) for gg in g]
        ctx.lidar_mesh_segment(ctx.prepare(inp, params, o), stream, "batched")
        torch.cuda.synchronize()
        paper[str(s)] = mean_scores(o, lp)
        log(f"  paper shape, interval {s}: {paper[str(s)]}")
    return {"measure": "edge points (a mesh join to another label / another surface), dilated by 1 lattice step; "
                       "precision, recall, F1 averaged over frames; truth = generator surface ids",
            "batch": batch, "paper_shape_32x1800": paper, "paper_shape_environments": n_env}


# The paper's own per-sweep times (Table 1: its C++ implementation on a
# 7th-generation Intel Core i5 with 8 GB DDR4; 32 rings x 1800 firings; mesh,
# normals and segmentation), quoted beside ours as context only.
PAPER_MS_PER_SWEEP = {5: 54.33, 10: 35.06, 15: 25.53}


def paper_shape_timing(lp, synth, torch, ctx, stream, reps=50):
    """The paper's sweep shape (32 x 1800, street scenes) at sampling intervals
    5, 10 and 15, inputs resident in HBM: one sweep per call (plain chain and
    graph replay, back to back: GPU time per sweep) and 64 sweeps per batched
    call (points/s)."""
    dev = torch.device("cuda", 0)
    params = lp.make_params(1.0, 60.0, (0.2, 0.2, 0.2))
    envs = synth.workload_frames("paper_32x1800", 8)
    res = {}

    def timed(prep, launch, n):
        for _ in range(3):
            ctx.lidar_mesh_segment(prep, stream, launch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            ctx.lidar_mesh_segment(prep, stream, launch)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n * 1e3

    for s in (5, 10, 15):
        geos = [lp.SensorGeometry(f.sensor.elevations(), f.sensor.n_azimuth, s, 1, f.sensor.az0) for f in envs]
        xs = [torch.from_numpy(f.xyz).to(dev) for f in envs]
        one_out = [lp.Outputs(geos[0], dev)]
        one = ctx.prepare([(xs[0], geos[0], None)], params, one_out)
        row = {"paper_ms_per_sweep": PAPER_MS_PER_SWEEP[s]}
        for launch in ("plain", "graph"):
            row[f"{launch}_ms_per_sweep"] = round(timed(one, launch, reps), 4)
        items = [(xs[k % 8], geos[k % 8], None) for k in range(64)]
        outs = [lp.Outputs(g, dev) for _, g, _ in items]
        batch = ctx.prepare(items, params, outs)
        ms = timed(batch, "batched", reps)
        row["batched64_points_per_s"] = round(sum(int(x.shape[0]) for x, _, _ in items) / (ms * 1e-3), 1)
        res[str(s)] = row
        log(f"  paper shape, interval {s}: {row}")
    return {"workload": "32 rings x 1800 firings, street scenes (8 environments), inputs resident in HBM",
            "paper_hardware": "C++ on a 7th-generation Intel Core i5, 8 GB DDR4 (Table 1; context only)",
            "intervals": res}


# The single-sweep configurations timed beside the batch: (name, workload, sampling interval s)
CONFIGS = (("C1", "c1_16x1800", 1), ("C2", "c2_64x2048", 1), ("C2", "c2_64x2048", 2),
           ("C2", "c2_64x2048", 4), ("C4", "c4_128x4096", 2))


def _same_outputs(a, b):
    """Two calls' outputs of one frame are equal: counts, and the vertices,
    normals, labels, vertex points and triangles they cover (the buffers are
    allocated at capacity; what lies past the counts is never written)."""
    import torch
    x, y = a.trimmed(), b.trimmed()
    if x["counts"] != y["counts"]:
        return False
    return all(torch.equal(x[k], y[k]) for k in ("vertices", "normals", "labels", "vertex_point", "triangles"))


def _timed(fn):
    t = time.perf_counter()
    fn()
    return time.perf_counter() - t


def path_bytes(N, V, T):
    """Algorithmic bytes of the whole path: xyz of every input point in; vertices,
    normals, labels, vertex_point and triangles out."""
    return 12 * N + 12 * V + 12 * V + 4 * V + 4 * V + 12 * T


def config_legs(lp, synth, torch, reps=200, lat_reps=100):
    """Each single-sweep configuration on its own, one sweep per call, inputs
    resident in HBM, in the plain form (one kernel chain) and as a graph replay:
    points/s of calls enqueued back to back (host clock), the GPU time of each
    call (HIP events on the launch stream, p50/p99), the latency of one call at a
    time (host call until its stream has finished, p50/p99) and the algorithmic
    bytes over the GPU time as a fraction of the HBM peak.  (The oracle's rate
    on the same sweeps is timed in the CPU-baseline leg.)"""
    import numpy as np
    from paper_2005_02704_amd import autotune
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    params = lp.make_params(1.0, 60.0, (0.2, 0.2, 0.2))
    res = {}
    for cname, wname, s in CONFIGS:
        f = synth.workload_frames(wname)[0]
        g = lp.SensorGeometry(f.sensor.elevations(), f.sensor.n_azimuth, s, 1, f.sensor.az0)
        ctx = lp.LidarContext(0)
        shape = autotune.apply(ctx, [g])
        out = lp.Outputs(g, dev)
        prep = ctx.prepare([(torch.from_numpy(f.xyz).to(dev), g, None)], params, [out])
        N = int(f.n_points)
        key = f"{cname}_{f.sensor.n_rings}x{f.sensor.n_azimuth}_s{s}"
        row = {"points": N, "launch_shape": shape}
        for launch in ("plain", "graph"):
            for _ in range(10):
                ctx.lidar_mesh_segment(prep, stream, launch)
            torch.cuda.synchronize()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            t0 = time.perf_counter()
            for a, b in evs:
                a.record(stream)
                ctx.lidar_mesh_segment(prep, stream, launch)
                b.record(stream)
            torch.cuda.synchronize()
            wall_ms = (time.perf_counter() - t0) * 1e3 / reps
            gpu = np.array([a.elapsed_time(b) for a, b in evs])
            lat = []
            for _ in range(lat_reps):
                t = time.perf_counter()
                ctx.lidar_mesh_segment(prep, stream, launch)
                stream.synchronize()
                lat.append((time.perf_counter() - t) * 1e3)
            V, T, K = (int(x) for x in out.counts.cpu())
            gpu_mean = float(gpu.mean())
            alg = path_bytes(N, V, T)
            row[launch] = {"points_per_s": round(N / (wall_ms * 1e-3), 1),
                           "gpu_points_per_s": round(N / (gpu_mean * 1e-3), 1),
                           "gpu_ms_p50": round(float(np.percentile(gpu, 50)), 5),
                           "gpu_ms_p99": round(float(np.percentile(gpu, 99)), 5),
                           "latency_ms_p50": round(float(np.percentile(lat, 50)), 5),
                           "latency_ms_p99": round(float(np.percentile(lat, 99)), 5),
                           "algorithmic_gbs": round(alg / (gpu_mean * 1e-3) / 1e9, 1),
                           "frac_of_hbm_peak": round(alg / (gpu_mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            row.update(vertices=V, triangles=T, segments=K, algorithmic_bytes=alg)
        ctx.close()
        res[key] = row
        log(f"  {key}: plain {row['plain']['points_per_s']:.3e} points/s (GPU p50 {row['plain']['gpu_ms_p50']:.4f} ms, "
            f"latency p99 {row['plain']['latency_ms_p99']:.4f} ms); graph {row['graph']['points_per_s']:.3e} points/s")
    return {"note": "one sweep per call, inputs resident in HBM; latency = host call until the stream has finished; "
                    "algorithmic bytes = 12 N + 32 V + 12 T over the mean GPU time of a call",
            "configs": res}


def rocm_version():
    """The ROCm release the library was built against, as installed."""
    try:
        with open("/opt/rocm/.info/version") as f:
            return f.read().strip()
    except OSError:
        return "unknown"


def cpu_model():
    """The host CPU's model name, as the kernel reports it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--cpu-seconds", type=float, default=16.0,
                    help="host time for the oracle baseline, half on one thread, half on --cpu-threads")
    ap.add_argument("--cpu-threads", type=int, default=16, help="threads of the all-core oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile-cells", type=int, default=0, help="0 = autotuned table / library default")
    ap.add_argument("--tile-threads", type=int, default=0, help="0 = autotuned table / library default")
    ap.add_argument("--grid", type=int, default=0, help="workgroups per batched stage, 0 = library default")
    ap.add_argument("--served-launch", default="graph", choices=("graph", "batched"),
                    help="launch form of the served run's groups")
    ap.add_argument("--served-seconds", type=float, default=60.0,
                    help="length of the served run (8 sensors, 10-20 Hz Poisson); 0 = skip")
    ap.add_argument("--in-flight", type=int, default=2,
                    help="also time the batched form with this many batches in flight (1 = skip)")
    ap.add_argument("--in-flight-launch", default="batched", help="launch forms timed in flight (batched, graph)")
    ap.add_argument("--in-flight-shape", default="",
                    help='launch shape of the batches in flight, as JSON ({"grid": G, "tile_cells": C, '
                         '"tile_threads": T, "stage_grids": {stage: G}}); default: the autotuned table')
    ap.add_argument("--forms", default="graph,batched,plain",
                    help="launch forms to time (graph is always timed: it gives value)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the single-sweep configurations (16x1800; 64x2048 at s = 1, 2, 4; 128x4096 at s = 2)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the edge-score leg and the timing at the paper's sweep shape")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (3 times), as the yardstick "
                         "for HBM byte counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: frames are independent, so a multi-GPU run is one "
              "single-GPU run per device; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2005_02704_amd as lp
    import synth

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {args.copy_calibration} MiB device copy done")
        del src, dst

    log(f"generating {args.frames} sweeps (seed {args.seed})")
    t0 = time.time()
    frames = synth.batch_frames(args.frames, args.seed)
    N = sum(f.n_points for f in frames)
    log(f"  {N} points in {time.time() - t0:.1f}s")

    dev = torch.device("cuda", 0)
    ctx = lp.LidarContext(0)
    params = lp.make_params(1.0, 60.0, (0.2, 0.2, 0.2))
    geos = [lp.SensorGeometry(f.sensor.elevations(), f.sensor.n_azimuth, 1, 1, f.sensor.az0) for f in frames]
    if args.grid or args.tile_cells or args.tile_threads:
        shape = {"grid": args.grid, "tile_cells": args.tile_cells, "tile_threads": args.tile_threads}
        ctx.set_tuning(args.grid, args.tile_cells, args.tile_threads)
        shape_src = "command line"
    else:
        from paper_2005_02704_amd import autotune
        shape = autotune.apply(ctx, geos)
        shape_src = f"autotuned table, class {autotune.batch_class(geos)}"
    n_flight = args.in_flight
    if args.in_flight_shape:
        if_shape = json.loads(args.in_flight_shape)
        if_shape.setdefault("stage_grids", {})
    elif shape_src == "command line":
        if_shape = shape
    else:
        if_shape = autotune.lookup_in_flight(geos)
    log(f"launch shape {shape} ({shape_src})")
    inputs = [(torch.from_numpy(f.xyz).to(dev), g, None) for f, g in zip(frames, geos)]
    outs = [lp.Outputs(g, dev) for g in geos]
    prep = ctx.prepare(inputs, params, outs)
    stream = torch.cuda.current_stream(dev)

    host_ms = {}

    def run(launch, steps, warmup, lanes=None, name=None):
        # W warmup steps, and at least half a second of this form, so clocks settle.
        # lanes: [(ctx, prepared call, stream), ...] used in turn, one step each, so
        # that many batches are in flight (each with its own workspace and outputs)
        lanes = lanes or [(ctx, prep, stream)]
        name = name or launch
        t_w = time.perf_counter()
        n_w = 0
        while n_w < warmup or time.perf_counter() - t_w < 0.5:
            c, pr, st = lanes[n_w % len(lanes)]
            c.lidar_mesh_segment(pr, st, launch)
            n_w += 1
            if n_w % 8 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(steps):
            c, pr, st = lanes[k % len(lanes)]
            c.lidar_mesh_segment(pr, st, launch)
        host_ms[name] = (time.perf_counter() - t) * 1000.0 / steps
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1000.0 / steps

    log("timing graph replays")
    ms_graph = run("graph", args.steps, args.warmup)
    counts = np.array([[int(x) for x in o.counts.cpu()] for o in outs])
    V, T = int(counts[:, 0].sum()), int(counts[:, 1].sum())
    log(f"  graph: {ms_graph:.3f} ms/step (host enqueue {host_ms['graph']:.3f} ms/step)  V={V} T={T}")
    forms = {"graph": {"points_per_s": round(N / (ms_graph * 1e-3), 1), "ms_per_step": round(ms_graph, 4),
                       "launch_shape": shape}}
    for form in ("batched", "plain"):
        if form not in args.forms.split(","):
            continue
        log(f"timing {form} launches")
        ms = run(form, args.steps, args.warmup)
        log(f"  {form}: {ms:.3f} ms/step (host enqueue {host_ms[form]:.3f} ms/step)")
        forms[form] = {"points_per_s": round(N / (ms * 1e-3), 1), "ms_per_step": round(ms, 4), "launch_shape": shape}
    if n_flight > 1 and "batched" in args.forms.split(","):
        # the batched form with several batches in flight: each step is still one
        # whole call over the batch, on one of `in_flight` contexts (workspace and
        # outputs of its own) and streams, taken in turn, so one batch's
        # latency-bound labelling stages overlap the next batch's mesh stages
        for launch in args.in_flight_launch.split(","):
            name = f"{launch}_x{n_flight}"
            log(f"timing {launch} launches, {n_flight} batches in flight, launch shape {if_shape}")
            extra = []
            for _ in range(n_flight):
                c2 = lp.LidarContext(0)
                from paper_2005_02704_amd import autotune
                autotune.set_shape(c2, if_shape)
                o2 = [lp.Outputs(g, dev) for g in geos]
                extra.append((c2, c2.prepare(inputs, params, o2), torch.cuda.Stream(dev), o2))
            torch.cuda.synchronize()   # the new outputs' fills are done before the lanes' streams use them
            ms = run(launch, args.steps, args.warmup, [(c2, p2, s2) for c2, p2, s2, _ in extra], name)
            same = all(_same_outputs(a, b) for c2, p2, s2, o2 in extra for a, b in zip(outs, o2))
            log(f"  {name}: {ms:.3f} ms/step (host enqueue {host_ms[name]:.3f} ms/step), "
                f"outputs as one in flight: {same}")
            if not same:
                raise RuntimeError("batches in flight gave other outputs than one batch alone")
            forms[name] = {"points_per_s": round(N / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
                           "launch_shape": if_shape}
            for c2, _, _, _ in extra:
                c2.close()
            del extra
    # roofline kernel: per-stage HIP events on the launch stream over K batched steps.
    # k_geom moves most of the path's algorithmic bytes (the kept points in; the
    # vertices, normals, vertex points and triangles out), so the roofline is its.
    log("timing stages with HIP events")
    ctx.stage_times()
    ctx.set_profiling(True)
    for _ in range(args.steps):
        ctx.lidar_mesh_segment(prep, stream, "batched")
    torch.cuda.synchronize()
    st = ctx.stage_times()
    ctx.set_profiling(False)
    per_launch = {k: ms / n for k, (ms, n) in st.items() if n}
    dom = "geom"
    dom_ms = per_launch[dom]
    dom_bytes = stage_bytes(dom, N, V, T)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    log("  stages (ms/launch): " + ", ".join(f"{k} {v:.4f}" for k, v in per_launch.items()))

    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{STAGE_KERNEL[dom]}.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            tr = json.load(f)
        if tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("frames") == args.frames \
                and tr.get("seed") == args.seed:
            traffic = tr.get("hbm_bytes_per_launch")

    roofline = {"bound": "hbm", "kernel": STAGE_KERNEL[dom], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": dom_bytes, "avg_launch_ms": round(dom_ms, 5),
                "stage_ms": {k: round(v, 5) for k, v in per_launch.items()}}
    # value: the fastest form that serves whole batches (graph replay, batched
    # launches, or batched launches with several batches in flight)
    best = max((f for f in forms if f != "plain"), key=lambda f: forms[f]["points_per_s"])
    ms_best = forms[best]["ms_per_step"]
    alg_path = path_bytes(N, V, T)
    path_gbs = alg_path / (ms_best * 1e-3) / 1e9
    roofline["path"] = {"algorithmic_bytes_per_step": alg_path, "ms_per_step": round(ms_best, 5),
                        "achieved": round(path_gbs, 1), "frac": round(path_gbs / HBM_PEAK_GBS, 4),
                        "launch": best}

    configs = None
    if not args.no_configs:
        log("single-sweep configurations")
        configs = config_legs(lp, synth, torch)

    accuracy = paper_timing = None
    if not args.no_accuracy:
        log("edge scores")
        accuracy = accuracy_run(args, lp, synth, torch, ctx, frames, geos, stream)
        log("the paper's sweep shape")
        paper_timing = paper_shape_timing(lp, synth, torch, ctx, stream)

    served = served_pool = None
    if args.served_seconds > 0:
        served, served_pool = served_run(args, lp, synth, torch)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        half = args.cpu_seconds / 2
        # single thread: the sweeps in order until half the time is spent
        log(f"timing the oracle on the host: one thread for ~{half:.0f}s")
        done_1, n_1 = 0, 0
        t = time.perf_counter()
        for f in frames:
            oracle.mesh_segment_frame(f)
            done_1 += f.n_points
            n_1 += 1
            if time.perf_counter() - t > half:
                break
        rate_1 = done_1 / (time.perf_counter() - t)
        # every core: one sweep per task (the oracle is C called through ctypes,
        # which releases the interpreter lock), the batch repeated until the
        # other half of the time is spent
        threads = max(1, min(args.cpu_threads, os.cpu_count() or 1))
        log(f"timing the oracle on the host: {threads} threads for ~{half:.0f}s")
        done_n, n_n = 0, 0
        t = time.perf_counter()
        with ThreadPoolExecutor(threads) as pool:
            while time.perf_counter() - t < half:
                for n in pool.map(lambda f: (oracle.mesh_segment_frame(f), f.n_points)[1], frames):
                    done_n += n
                    n_n += 1
        rate_n = done_n / (time.perf_counter() - t)
        cpu = {"value": round(rate_n, 1), "unit": "points/s", "cores": threads, "kind": "oracle",
               "sample": f"{n_n} sweeps ({done_n} points) of the same batch on {threads} threads, one sweep per "
                         f"task; host has {os.cpu_count()} CPUs ({cpu_model()})",
               "single_thread_points_per_s": round(rate_1, 1),
               "single_thread_sample": f"first {n_1} of the {args.frames} sweeps ({done_1} points)"}
        log(f"  oracle: {rate_n:.0f} points/s on {threads} threads, {rate_1:.0f} points/s on one")
        if configs is not None:
            # each single-sweep configuration on one thread (best of two runs)
            per = {}
            for cname, wname, s_ in CONFIGS:
                f = synth.workload_frames(wname)[0]
                best_t = min(_timed(lambda: oracle.mesh_segment_frame(f, s=s_)) for _ in range(2))
                per[f"{cname}_{f.sensor.n_rings}x{f.sensor.n_azimuth}_s{s_}"] = round(f.n_points / best_t, 1)
            cpu["per_config_1_thread_points_per_s"] = per
        if served_pool is not None:
            # the served pool's sweeps one at a time on one thread: the latency a
            # host-only server would add per sweep, beside the served p50/p99
            ms = np.array([_timed(lambda: oracle.mesh_segment_frame(f)) * 1e3 for f in served_pool])
            cpu["served_pool_sweep_ms"] = {"p50": round(float(np.percentile(ms, 50)), 3),
                                           "p99": round(float(np.percentile(ms, 99)), 3),
                                           "sweeps": len(served_pool)}

    value = N / (ms_best * 1e-3)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_best, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched {args.frames} uneven street sweeps (rings 16/32/64/128, "
                               f"azimuth 1024/2048/4096, s=1)", "frames": args.frames,
                   "points_per_step": N, "vertices_per_step": V, "triangles_per_step": T,
                   "launch": best, "seed": args.seed, "launch_shape": forms[best]["launch_shape"],
                   "launch_shape_source": shape_src, "rocm": rocm_version(),
                   "device": torch.cuda.get_device_name(0),
                   "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", ""),
                   "compute_units": torch.cuda.get_device_properties(0).multi_processor_count},
        "forms": forms,
        "vertices_per_s": round(V / (ms_best * 1e-3), 1),
        "path_algorithmic_gbs": round(path_gbs, 1),
        "roofline": roofline,
        "single_sweep": configs,
        "served": served,
        "accuracy": accuracy,
        "paper_shape_timing": paper_timing,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
