"""Autotuner for the launch shape of the batched path.

The shape of a call -- workgroups per grid-stride stage, cells per lattice tile
and threads per tile workgroup -- changes only the speed, never the results
(the kernels are written so that every shape produces identical outputs; the
GPU tests check this).  The best shape depends on the batch: few wide frames
favour big tiles, many narrow ones more workgroups.  This module

  * classifies a batch (ring count, sampled width, number of frames),
  * times every candidate shape on a prepared batch with HIP events on the
    launch stream (the whole chain, median of a few replays),
  * keeps the winners in a JSON table (`tune_table.json` next to this file),
  * and looks a batch's shape up in that table.

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
GRIDS = (1024, 2048, 4096)
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
    """Tuned shape for this batch, or the library default when its class is absent."""
    table = load_table() if table is None else table
    entry = table.get(batch_class(geometries))
    if not entry:
        return dict(DEFAULT)
    return {k: int(entry[k]) for k in ("grid", "tile_cells", "tile_threads")}


def apply(ctx, geometries, table: dict | None = None) -> dict:
    """Set the tuned shape of this batch on a LidarContext; returns it."""
    shape = lookup(geometries, table)
    ctx.set_tuning(shape["grid"], shape["tile_cells"], shape["tile_threads"])
    return shape


def time_shape(ctx, prepared, stream, shape, launch="graph", reps=12, warm=3) -> float:
    """Median milliseconds of one call with this shape (events on the launch stream)."""
    import torch
    ctx.set_tuning(shape["grid"], shape["tile_cells"], shape["tile_threads"])
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
    ctx.set_tuning(0, 0, 0)
    return best[0], results


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
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import paper_2005_02704_amd as lp
    import synth

    def log(m):
        print(m, file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    ctx = lp.LidarContext(0)
    params = lp.make_params(1.0, 60.0, (0.2, 0.2, 0.2))
    classes = {}
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
            classes[key] = {**best, "ms": round(best_ms, 5), "default_ms": round(default_ms, 5), "workload": name}
    ctx.close()
    with open(args.out, "w") as f:
        json.dump({"device": torch.cuda.get_device_name(0), "classes": classes}, f, indent=1, sort_keys=True)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
