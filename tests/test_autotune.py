"""The launch-shape autotuner's host side: batch classes, the committed table,
and that every shape it may choose is one the library accepts."""
import numpy as np

import paper_2005_02704_amd as lp
from paper_2005_02704_amd import autotune


def _geo(h, w, s=1):
    return lp.SensorGeometry(np.linspace(0.2, -0.3, h), w, s)


def test_batch_class_buckets():
    assert autotune.batch_class([_geo(16, 1800)]) == "H16-W2048-F1"
    assert autotune.batch_class([_geo(64, 2048, 2)]) == "H64-W1024-F1"
    assert autotune.batch_class([_geo(16, 1024), _geo(128, 4096)] * 10) == "H128-W4096-F64"
    assert autotune.batch_class([_geo(100, 9000)] * 300) == "H128-W16384-F512"


def test_lookup_falls_back_to_the_default():
    assert autotune.lookup([_geo(7, 333)], table={}) == {**autotune.DEFAULT, "stage_grids": {}}


def test_lookup_returns_stage_grids():
    key = autotune.batch_class([_geo(16, 1800)])
    table = {key: {"grid": 2048, "tile_cells": 512, "tile_threads": 256, "ms": 1.0, "default_ms": 1.0,
                   "stage_grids": {"bin": 1536, "geom": 6144}}}
    shape = autotune.lookup([_geo(16, 1800)], table=table)
    assert shape == {"grid": 2048, "tile_cells": 512, "tile_threads": 256,
                     "stage_grids": {"bin": 1536, "geom": 6144}}


def test_committed_table_holds_supported_shapes():
    table = autotune.load_table()
    assert table, "tune_table.json is missing"
    shapes = {(c, t) for c, t in autotune.TILE_SHAPES}
    for key, entry in table.items():
        assert (entry["tile_cells"], entry["tile_threads"]) in shapes, key
        assert entry["grid"] in autotune.GRIDS
        assert entry["ms"] <= entry["default_ms"] + 1e-9
        from paper_2005_02704_amd.lidarseg import STAGES
        for stage, g in entry.get("stage_grids", {}).items():
            assert stage in STAGES and g in autotune.STAGE_GRIDS, (key, stage, g)
        f = entry.get("in_flight")
        if f:
            assert (f["tile_cells"], f["tile_threads"]) in shapes, key
            assert f["grid"] > 0 and f["batches"] >= 2
            for stage, g in f.get("stage_grids", {}).items():
                assert stage in STAGES and g > 0, (key, stage, g)
    # the benchmark batch has an entry, and a shape for two batches in flight
    assert "H128-W4096-F64" in table
    assert "in_flight" in table["H128-W4096-F64"]


def test_lookup_in_flight():
    geos = [_geo(16, 1800)]
    key = autotune.batch_class(geos)
    one = {"grid": 2048, "tile_cells": 512, "tile_threads": 256, "ms": 1.0, "default_ms": 1.0}
    assert autotune.lookup_in_flight(geos, table={key: one}) == {**{k: one[k] for k in ("grid", "tile_cells",
                                                                                          "tile_threads")},
                                                                 "stage_grids": {}}
    two = {**one, "in_flight": {"grid": 512, "tile_cells": 2048, "tile_threads": 512, "batches": 2,
                                "stage_grids": {"geom": 768}}}
    assert autotune.lookup_in_flight(geos, table={key: two}) == {"grid": 512, "tile_cells": 2048,
                                                                 "tile_threads": 512, "stage_grids": {"geom": 768}}


def test_candidates_cover_every_shape_and_grid():
    c = autotune.candidates()
    assert len(c) == len(autotune.TILE_SHAPES) * len(autotune.GRIDS)
    assert len({tuple(sorted(x.items())) for x in c}) == len(c)


def test_in_flight_descent_picks_the_fastest_and_keeps_only_real_gains():
    """The in-flight tuner's coordinate descent on a made-up cost: the grid is
    chosen first, then a stage count that is more than 0.5 % faster is kept, and
    one that is faster by less is not; the one-batch shape wins when nothing
    beats it."""
    base = {"grid": 1536, "tile_cells": 2048, "tile_threads": 512, "stage_grids": {"geom": 3072}}

    def cost(shape):
        g = shape["grid"]
        ms = 0.40 + abs(g - 512) * 1e-5
        sg = shape["stage_grids"]
        if sg.get("geom") == 768:
            ms -= 0.01          # a real gain
        if sg.get("cc") == 1536:
            ms -= 0.0005        # below the 0.5 % bar
        return ms

    shape, ms, base_ms = autotune.tune_in_flight(None, None, None, base, timer=cost)
    assert shape == {"grid": 512, "tile_cells": 2048, "tile_threads": 512, "stage_grids": {"geom": 768}}
    assert abs(ms - 0.39) < 1e-9 and abs(base_ms - cost(base)) < 1e-12
    shape, ms, base_ms = autotune.tune_in_flight(None, None, None, base, timer=lambda s: 0.3 if s is base else 0.5)
    assert shape is base and ms == base_ms == 0.3
