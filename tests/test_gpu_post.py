"""GPU parity of the steps after Algorithm 1 and of the cosine test.

Every input point's label (back-fill along the sweep), segment removal and the
cosine similarity test, through the C ABI against the FP64 oracle: bit-exact on
the oracle's own normals and on margin-cleared sweeps.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import check_geometry, margin_clear_cos, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

COS = float(np.cos(np.radians(12.0)))


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_02704_amd as lp
    c = lp.LidarContext(0)
    yield c
    c.close()


CASES = [("paper_32x1800", 5, 1), ("paper_32x1800", 15, 1), ("c2_64x2048", 2, 1), ("c2_64x2048", 4, 0),
         ("c4_128x4096", 2, 1), ("c1_16x1800", 1, 1)]


@pytest.mark.parametrize("name,s,wrap", CASES)
def test_point_labels_bit_exact(ctx, name, s, wrap):
    f = synth.workload_frames(name)[0]
    print(f"case {name} s={s} wrap={wrap} N={f.n_points}", flush=True)
    r = run_oracle(f.xyz, f.sensor, s, wrap, point_labels=True)
    g = run_gpu(ctx, [(f.xyz, f.sensor, s, wrap, r.normals)], point_labels=True)[0]
    assert np.array_equal(g["labels"], r.labels)
    assert np.array_equal(g["point_labels"], r.point_labels)


@pytest.mark.parametrize("m", [2, 3, 10])
@pytest.mark.parametrize("name,s", [("c1_16x1800", 1), ("paper_32x1800", 5)])
def test_segment_removal_bit_exact(ctx, name, s, m):
    f = synth.workload_frames(name)[0]
    r = run_oracle(f.xyz, f.sensor, s, min_segment=m, point_labels=True)
    g = run_gpu(ctx, [(f.xyz, f.sensor, s, 1, r.normals)], min_segment=m, point_labels=True)[0]
    assert g["counts"][2] == r.counts[2]
    assert np.array_equal(g["labels"], r.labels)
    assert np.array_equal(g["point_labels"], r.point_labels)


@pytest.mark.parametrize("name,s", [("c1_16x1800", 1), ("c2_64x2048", 2), ("c4_128x4096", 2)])
def test_cosine_labels_on_oracle_normals(ctx, name, s):
    f = synth.workload_frames(name)[0]
    r = run_oracle(f.xyz, f.sensor, s, predicate=1, cos_min=COS)
    g = run_gpu(ctx, [(f.xyz, f.sensor, s, 1, r.normals)], predicate=1, cos_min=COS)[0]
    assert g["counts"][2] == r.counts[2]
    assert np.array_equal(g["labels"], r.labels)


@pytest.mark.parametrize("name,s", [("c1_16x1800", 1), ("c2_64x2048", 2)])
def test_cosine_margin_cleared_end_to_end(ctx, name, s):
    f = synth.workload_frames(name)[0]
    xyz = margin_clear_cos(f.xyz, f.sensor, COS, s)
    print(f"case {name} s={s}: {f.n_points - xyz.shape[0]} points dropped by margin clearing", flush=True)
    r = run_oracle(xyz, f.sensor, s, predicate=1, cos_min=COS, point_labels=True, min_segment=4)
    g = run_gpu(ctx, [(xyz, f.sensor, s, 1, None)], predicate=1, cos_min=COS, point_labels=True, min_segment=4)[0]
    check_geometry(g, r)
    assert np.array_equal(g["labels"], r.labels)
    assert np.array_equal(g["point_labels"], r.point_labels)


def test_post_stage_in_every_launch_form(ctx):
    frames = synth.batch_frames(8, 321)
    refs = [run_oracle(f.xyz, f.sensor, 1, min_segment=3, point_labels=True) for f in frames]
    items = [(f.xyz, f.sensor, 1, 1, r.normals) for f, r in zip(frames, refs)]
    for launch in ("plain", "batched", "graph", "graph"):
        got = run_gpu(ctx, items, launch=launch, min_segment=3, point_labels=True)
        for r, g in zip(refs, got):
            assert np.array_equal(g["labels"], r.labels), launch
            assert np.array_equal(g["point_labels"], r.point_labels), launch
    # and a call without the stage afterwards (the graph is captured again)
    got = run_gpu(ctx, items, launch="graph")
    ref0 = [run_oracle(f.xyz, f.sensor, 1) for f in frames]
    for r, g in zip(ref0, got):
        assert np.array_equal(g["labels"], r.labels)


def test_cosine_and_removal_in_batched_and_graph_forms(ctx):
    """The cosine test, segment removal and point labels on a batch of uneven
    sweeps in the batched and graph forms (labels on the oracle's normals, so
    bit-exact), replayed twice."""
    frames = synth.batch_frames(6, 4242)
    refs = [run_oracle(f.xyz, f.sensor, 1, predicate=1, cos_min=COS, min_segment=3, point_labels=True)
            for f in frames]
    items = [(f.xyz, f.sensor, 1, 1, r.normals) for f, r in zip(frames, refs)]
    for launch in ("batched", "graph", "graph"):
        got = run_gpu(ctx, items, launch=launch, predicate=1, cos_min=COS, min_segment=3, point_labels=True)
        for k, (g, r) in enumerate(zip(got, refs)):
            assert g["counts"][2] == r.counts[2], (launch, k)
            assert np.array_equal(g["labels"], r.labels), (launch, k)
            assert np.array_equal(g["point_labels"], r.point_labels), (launch, k)
