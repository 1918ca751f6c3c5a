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


def served_run(args, lp, synth, torch):
    """8 simulated sensors (rings 16/32/64/128, widths 1024/2048/4096, 10-20 Hz
    Poisson arrivals) through the continuous-batching server; then the same pool
    with every request arriving at once (capacity), served in groups and, for
    comparison, one sweep per call with plain per-frame launches."""
    from paper_2005_02704_amd.serve import GpuExecutor, Request, Server, poisson_schedule
    sensors = synth.served_sensors(8)
    n_pool = 3
    log(f"served: generating {8 * n_pool} pool sweeps")
    pool = [[synth.make_frame(s, "street", synth.frame_seed(9000 + q, k), sigma=0.01, dropout=0.10)
             for k in range(n_pool)] for q, (s, _) in enumerate(sensors)]
    geos = [lp.SensorGeometry(s.elevations(), s.n_azimuth, 1, 1, s.az0) for s, _ in sensors]
    pinned = [[torch.from_numpy(f.xyz).pin_memory() for f in row] for row in pool]

    def make(rid, s, k, t):
        return Request(rid, s, pinned[s][k], pool[s][k].n_points, t)

    budget = 1 << 30
    ex = GpuExecutor(geos, n_slots=3, launch=args.served_launch)
    # warm the slots (workspace growth, graph capture) before timing
    warm = Server(ex, budget_bytes=budget, max_batch=16)
    warm.run_schedule([(0.0, q, 0) for q in range(8)] * 3, make)
    srv = Server(ex, budget_bytes=budget, max_batch=16, timeout_s=1.0)
    sched = poisson_schedule([r for _, r in sensors], args.served_seconds, seed=args.seed, n_payloads=n_pool)
    log(f"served: {len(sched)} sweeps over {args.served_seconds:.0f}s")
    wall = srv.run_schedule(sched, make)
    st = srv.stats(wall)
    log(f"  p50 {st['p50_ms']:.2f} ms  p99 {st['p99_ms']:.2f} ms  {st['points_per_s']:.3e} points/s")
    burst = [(0.0, q % 8, (q // 8) % n_pool) for q in range(8 * 64)]
    # one untimed burst first: the buffer sets the larger groups need (device
    # outputs, pinned host copies) are allocated once, as a long-running server's are
    Server(ex, budget_bytes=budget, max_batch=64).run_schedule(burst, make)
    cap = Server(ex, budget_bytes=budget, max_batch=64)
    wall_c = cap.run_schedule(burst, make)
    stc = cap.stats(wall_c)
    log(f"  capacity: {stc['points_per_s']:.3e} points/s ({stc['requests']} sweeps at once)")
    ex.close()
    # the same burst served one sweep per call with plain per-frame launches
    ex_p = GpuExecutor(geos, n_slots=3, launch="plain")
    Server(ex_p, budget_bytes=budget, max_batch=1).run_schedule(burst, make)
    cap_p = Server(ex_p, budget_bytes=budget, max_batch=1)
    stp = cap_p.stats(cap_p.run_schedule(burst, make))
    log(f"  capacity, one sweep per plain call: {stp['points_per_s']:.3e} points/s")
    ex_p.close()
    keep = ("requests", "failed", "points_per_s", "p50_ms", "p99_ms", "max_ms", "mean_batch",
            "max_slots_in_flight", "peak_device_bytes")
    return {"workload": "8 sensors, rings 16/32/64/128, azimuth 1024/2048/4096, 10-20 Hz Poisson, "
                        f"{args.served_seconds:.0f}s, budget 1 GiB, 3 slots, {args.served_launch} launches, "
                        "1 s watchdog per group",
            **{k: (round(st[k], 3) if isinstance(st[k], float) else st[k]) for k in keep},
            "latency": "host arrival to labels/vertex_point/counts in pinned host memory",
            "capacity_points_per_s": round(stc["points_per_s"], 1),
            "capacity_mean_batch": round(stc["mean_batch"], 2),
            "capacity_plain_one_sweep_per_call_points_per_s": round(stp["points_per_s"], 1)}


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
    ap.add_argument("--served-seconds", type=float, default=10.0,
                    help="length of the served run (8 sensors, 10-20 Hz Poisson); 0 = skip")
    ap.add_argument("--in-flight", type=int, default=2,
                    help="also time the batched form with this many batches in flight (1 = skip)")
    ap.add_argument("--forms", default="graph,batched,plain",
                    help="launch forms to time (graph is always timed: it gives value)")
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
    if_shape, n_flight = shape, args.in_flight
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
        name = f"batched_x{n_flight}"
        log(f"timing batched launches, {n_flight} batches in flight, launch shape {if_shape}")
        extra = []
        for _ in range(n_flight):
            c2 = lp.LidarContext(0)
            from paper_2005_02704_amd import autotune
            autotune.set_shape(c2, if_shape)
            o2 = [lp.Outputs(g, dev) for g in geos]
            extra.append((c2, c2.prepare(inputs, params, o2), torch.cuda.Stream(dev), o2))
        ms = run("batched", args.steps, args.warmup, [(c2, p2, s2) for c2, p2, s2, _ in extra], name)
        same = all(torch.equal(a.labels, b.labels) and torch.equal(a.counts, b.counts)
                   for c2, p2, s2, o2 in extra for a, b in zip(outs, o2))
        log(f"  {name}: {ms:.3f} ms/step (host enqueue {host_ms[name]:.3f} ms/step), outputs as one in flight: {same}")
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
    alg_path = 12 * N + 12 * V + 12 * V + 4 * V + 4 * V + 12 * T   # whole path, as in the byte model
    path_gbs = alg_path / (ms_best * 1e-3) / 1e9

    accuracy = paper_timing = None
    if not args.no_accuracy:
        log("edge scores")
        accuracy = accuracy_run(args, lp, synth, torch, ctx, frames, geos, stream)
        log("the paper's sweep shape")
        paper_timing = paper_shape_timing(lp, synth, torch, ctx, stream)

    served = None
    if args.served_seconds > 0:
        served = served_run(args, lp, synth, torch)

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
        "served": served,
        "accuracy": accuracy,
        "paper_shape_timing": paper_timing,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
