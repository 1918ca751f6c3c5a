"""Autotuner for the launch shape of the batched path.

The shape of a call -- workgroups per grid-stride stage, cells per lattice tile
and threads per tile workgroup -- changes only the speed, never the results
(the kernels are written so that every shape produces identical outputs; the
GPU tests check this).  The best shape depends on the batch: few wide frames
favour big tiles, many narrow ones more workgroups.  This module

  * classifies a batch (ring count, sampled width, number of frames),
  * times every candidate shape on a prepared batch with HIP events on the
    launch stream (the whole chain, median of a few replays),
  * then, in the winning shape, times each stage's kernel (HIP events) at other
    workgroup counts and keeps a stage's own count where it is faster, when the
    whole call is faster with them,
  * keeps the winners in a JSON table (`tune_table.json` next to this file),
  * and looks a batch's shape up in that table.

A class may also carry an "in_flight" shape, used when several batches of it
run at once on their own contexts and streams: there each stage shares the GPU
with the other batch's stages, and fewer workgroups per stage overlap better.
`python -m paper_2005_02704_amd.autotune --in-flight 2` tunes it for the
benchmark batch (fresh contexts for every candidate, shaped before any call and
synchronised before the next); a rebuild of the table keeps it.

Run `python -m paper_2005_02704_amd.autotune` on the GPU to rebuild the table
for the standard synthetic workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "tune_table.json")

TILE_SHAPES = ((1024, 256), (512, 256), (2048, 256), (1024, 512), (2048, 512))
GRIDS = (1024, 1536, 2048, 3072, 4096, 6144)
DEFAULT = {"grid": 0, "tile_cells": 1024, "tile_threads": 256}


def _bucket(x, edges):
    for e in edges:
        if x <= e:
            return e
    return edges[-1] * 2


def batch_class(geometries) -> str:
    """Key of a batch: largest ring count, largest sampled width and frame count,
    each rounded up to a bucket edge."""
    h = max(g.n_rings for g in geometries)
    w = max(g.n_cols for g in geometries)
    n = len(geometries)
    return f"H{_bucket(h, (16, 32, 64, 128))}-W{_bucket(w, (1024, 2048, 4096, 8192))}-F{_bucket(n, (1, 4, 16, 64, 256))}"


def load_table(path: str = TABLE_PATH) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f).get("classes", {})


def lookup(geometries, table: dict | None = None) -> dict:
    """Tuned shape for this batch, or the library default when its class is absent:
    grid, tile_cells, tile_threads and stage_grids ({stage: workgroups})."""
    table = load_table() if table is None else table
    entry = table.get(batch_class(geometries))
    if not entry:
        return {**DEFAULT, "stage_grids": {}}
    shape = {k: int(entry[k]) for k in ("grid", "tile_cells", "tile_threads")}
    shape["stage_grids"] = {k: int(v) for k, v in entry.get("stage_grids", {}).items()}
    return shape


def lookup_in_flight(geometries, table: dict | None = None) -> dict:
    """Shape for several batches of this class in flight at once (each on its
    own context and stream): the class's "in_flight" entry when it has one,
    else its one-batch shape."""
    table = load_table() if table is None else table
    entry = (table.get(batch_class(geometries)) or {}).get("in_flight")
    if not entry:
        return lookup(geometries, table)
    shape = {k: int(entry[k]) for k in ("grid", "tile_cells", "tile_threads")}
    shape["stage_grids"] = {k: int(v) for k, v in entry.get("stage_grids", {}).items()}
    return shape


def set_shape(ctx, shape: dict) -> None:
    """Apply a shape (as lookup returns it) to a LidarContext."""
    from .lidarseg import STAGES
    ctx.set_tuning(shape["grid"], shape["tile_cells"], shape["tile_threads"])
    grids = shape.get("stage_grids", {})
    for stage in STAGES:
        ctx.set_stage_grid(stage, grids.get(stage, 0))


def apply(ctx, geometries, table: dict | None = None) -> dict:
    """Set the tuned shape of this batch on a LidarContext; returns it."""
    shape = lookup(geometries, table)
    set_shape(ctx, shape)
    return shape


def time_shape(ctx, prepared, stream, shape, launch="graph", reps=12, warm=3) -> float:
    """Median milliseconds of one call with this shape (events on the launch stream)."""
    import torch
    set_shape(ctx, shape)
    for _ in range(warm):
        ctx.lidar_mesh_segment(prepared, stream, launch)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.lidar_mesh_segment(prepared, stream, launch)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


STAGE_GRIDS = (256, 512, 1024, 1536, 2048, 3072, 4096, 6144, 8192)
TUNED_STAGES = ("bin", "count", "geom", "cc", "merge", "compress", "flatten", "label")


def stage_ms(ctx, prepared, stream, reps=10) -> dict:
    """Milliseconds per launch of every stage over `reps` batched calls (events)."""
    import torch
    for _ in range(2):
        ctx.lidar_mesh_segment(prepared, stream, "batched")
    torch.cuda.synchronize()
    ctx.stage_times()
    ctx.set_profiling(True)
    for _ in range(reps):
        ctx.lidar_mesh_segment(prepared, stream, "batched")
    torch.cuda.synchronize()
    st = ctx.stage_times()
    ctx.set_profiling(False)
    return {k: ms / n for k, (ms, n) in st.items() if n}


def tune_stage_grids(ctx, prepared, stream, shape, log=None) -> dict:
    """In `shape`, each tuned stage's workgroup count that beats its share of the
    grid by at least 2 % in that stage's own time; returns {stage: workgroups}."""
    set_shape(ctx, {**shape, "stage_grids": {}})
    base = stage_ms(ctx, prepared, stream)
    chosen = {}
    for stage in TUNED_STAGES:
        best_g, best = 0, base[stage]
        for g in STAGE_GRIDS:
            ctx.set_stage_grid(stage, g)
            ms = stage_ms(ctx, prepared, stream)[stage]
            if ms < best * 0.98:
                best_g, best = g, ms
        ctx.set_stage_grid(stage, best_g)
        if best_g:
            chosen[stage] = best_g
            if log:
                log(f"  stage {stage}: {best_g} workgroups, {best:.4f} ms (share of the grid {base[stage]:.4f} ms)")
    return chosen


def candidates():
    return [{"grid": g, "tile_cells": c, "tile_threads": t} for g in GRIDS for (c, t) in TILE_SHAPES]


def tune(ctx, prepared, stream, launch="graph", log=None):
    """Time every candidate; returns (best shape, [(shape, ms), ...])."""
    results = []
    for shape in candidates():
        ms = time_shape(ctx, prepared, stream, shape, launch)
        results.append((shape, ms))
        if log:
            log(f"  {shape} {ms:.4f} ms")
    best = min(results, key=lambda r: r[1])
    set_shape(ctx, {**DEFAULT, "stage_grids": {}})
    return best[0], results


def time_in_flight(inputs, geometries, params, shape, n_flight=2, steps=100, warm=6) -> float:
    """Milliseconds per batch with `n_flight` batches in flight at `shape`: that
    many fresh contexts, each with its own outputs and stream, take batched calls
    in turn (host clock over `steps` calls, fully synchronised before and after).
    The contexts are made, shaped and synchronised before any call, and closed
    after the last; nothing is re-shaped while another context runs."""
    import time
    import torch
    from . import lidarseg as lp
    dev = torch.device("cuda", 0)
    lanes = []
    try:
        for _ in range(n_flight):
            c = lp.LidarContext(0)
            set_shape(c, shape)
            outs = [lp.Outputs(g, dev) for g in geometries]
            lanes.append((c, c.prepare(inputs, params, outs), torch.cuda.Stream(dev), outs))
        torch.cuda.synchronize()   # the outputs' fills are done before the lanes' streams use them
        for k in range(warm):
            c, p, st, _ = lanes[k % n_flight]
            c.lidar_mesh_segment(p, st, "batched")
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(steps):
            c, p, st, _ = lanes[k % n_flight]
            c.lidar_mesh_segment(p, st, "batched")
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / steps
    finally:
        torch.cuda.synchronize()
        for c, _, _, _ in lanes:
            c.close()


IN_FLIGHT_GRIDS = (384, 512, 640, 768, 1024, 1536)
IN_FLIGHT_STAGE_GRIDS = {"geom": (768, 1024, 1536, 3072), "cc": (768, 1536), "bin": (768, 1536)}


def tune_in_flight(inputs, geometries, params, base_shape, n_flight=2, log=None, timer=None):
    """Shape for `n_flight` batches in flight, by coordinate descent from the
    one-batch shape's tile: the grid first, then each stage of
    IN_FLIGHT_STAGE_GRIDS in turn, a change kept only when it is 0.5 % faster
    (each shape timed three times, the fastest kept).  timer(shape) -> ms
    replaces time_in_flight (for tests).
    Returns (shape, ms, ms of the one-batch shape in flight)."""
    timer = timer or (lambda shape: time_in_flight(inputs, geometries, params, shape, n_flight))

    def run(shape):
        ms = min(timer(shape) for _ in range(3))
        if log:
            log(f"  in flight x{n_flight}: {shape} {ms:.4f} ms")
        return ms

    base_ms = run(base_shape)
    tile = {"tile_cells": base_shape["tile_cells"], "tile_threads": base_shape["tile_threads"]}
    best, best_ms = None, None
    for g in IN_FLIGHT_GRIDS:
        shape = {"grid": g, **tile, "stage_grids": {}}
        ms = run(shape)
        if best_ms is None or ms < best_ms:
            best, best_ms = shape, ms
    for stage, grids in IN_FLIGHT_STAGE_GRIDS.items():
        for g in grids:
            shape = {**best, "stage_grids": {**best["stage_grids"], stage: g}}
            ms = run(shape)
            if ms < best_ms * 0.995:
                best, best_ms = shape, ms
    if base_ms <= best_ms:
        return base_shape, base_ms, base_ms
    return best, best_ms, base_ms


def _workloads():
    """The batches the table is built for: the benchmark batch, served-style
    groups of a few sensors, and the single-frame workloads."""
    import synth
    out = [("batch64", synth.batch_frames(64, 2024))]
    out.append(("batch16", synth.batch_frames(16, 77)))
    out.append(("batch4", synth.batch_frames(4, 78)))
    for name in ("c1_16x1800", "c2_64x2048", "c4_128x4096", "paper_32x1800"):
        out.append((name, synth.workload_frames(name)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="rebuild the launch-shape table on the GPU")
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--in-flight", type=int, default=0, metavar="N",
                    help="only (re)tune the benchmark batch's shape for N batches in flight, keeping the rest")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import paper_2005_02704_amd as lp
    import synth

    def log(m):
        print(m, file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    params = lp.make_params(1.0, 60.0, (0.2, 0.2, 0.2))
    if args.in_flight > 1:
        classes = load_table(args.out)
        frames = synth.batch_frames(64, 2024)
        geos = [lp.SensorGeometry(f.sensor.elevations(), f.sensor.n_azimuth, 1, 1, f.sensor.az0) for f in frames]
        key = batch_class(geos)
        if key not in classes:
            raise SystemExit(f"no one-batch entry for {key}: tune the table first")
        inputs = [(torch.from_numpy(f.xyz).to(dev), g, None) for f, g in zip(frames, geos)]
        one = lookup(geos, classes)
        shape, ms, base_ms = tune_in_flight(inputs, geos, params, one, args.in_flight, log)
        classes[key]["in_flight"] = {**shape, "batches": args.in_flight, "ms": round(ms, 5),
                                     "one_batch_shape_ms": round(base_ms, 5)}
        log(f"{key}: in flight x{args.in_flight} {shape} {ms:.4f} ms (one-batch shape {base_ms:.4f} ms)")
        with open(args.out, "w") as f:
            json.dump({"device": torch.cuda.get_device_name(0), "classes": classes}, f, indent=1, sort_keys=True)
        log(f"wrote {args.out}")
        return
    ctx = lp.LidarContext(0)
    classes = {}
    previous = load_table(args.out)
    for name, frames in _workloads():
        s = synth.WORKLOADS[name]["s"][0] if name in synth.WORKLOADS else 1
        geos = [lp.SensorGeometry(f.sensor.elevations(), f.sensor.n_azimuth, s, 1, f.sensor.az0) for f in frames]
        key = batch_class(geos)
        inputs = [(torch.from_numpy(f.xyz).to(dev), g, None) for f, g in zip(frames, geos)]
        outs = [lp.Outputs(g, dev) for g in geos]
        prep = ctx.prepare(inputs, params, outs)
        log(f"{name}: class {key}, {len(frames)} frames")
        best, results = tune(ctx, prep, stream, "graph", log)
        ms = dict((json.dumps(sh, sort_keys=True), m) for sh, m in results)
        default_ms = ms[json.dumps({"grid": 1024, "tile_cells": 1024, "tile_threads": 256}, sort_keys=True)]
        best_ms = min(m for _, m in results)
        log(f"  best {best} {best_ms:.4f} ms (default {default_ms:.4f} ms)")
        if key not in classes or best_ms < classes[key]["ms"]:
            grids = tune_stage_grids(ctx, prep, stream, best, log)
            entry = {**best, "ms": round(best_ms, 5), "default_ms": round(default_ms, 5), "workload": name}
            if grids:
                # keep them only if the whole call (graph replay) is faster with them
                ms_g = min(time_shape(ctx, prep, stream, {**best, "stage_grids": grids}) for _ in range(2))
                ms_0 = min(time_shape(ctx, prep, stream, {**best, "stage_grids": {}}) for _ in range(2))
                log(f"  with stage grids {ms_g:.4f} ms, without {ms_0:.4f} ms")
                if ms_g < ms_0:
                    entry["stage_grids"] = grids
                    entry["ms"] = round(ms_g, 5)
            set_shape(ctx, {**DEFAULT, "stage_grids": {}})
            if "in_flight" in previous.get(key, {}):
                entry["in_flight"] = previous[key]["in_flight"]
            classes[key] = entry
    ctx.close()
    with open(args.out, "w") as f:
        json.dump({"device": torch.cuda.get_device_name(0), "classes": classes}, f, indent=1, sort_keys=True)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
