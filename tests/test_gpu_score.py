"""GPU parity of the edge scores (the evaluation of Section 3: segment edge
points against ground-truth surface edge points, each dilated by R lattice
steps), through the C ABI against the FP64 oracle.

  * on the oracle's own normals the labels are bit-exact, so the four counts
    must equal the oracle's scores of the oracle's labels;
  * on raw sweeps (GPU normals) the counts must equal the oracle's scores of
    the GPU's own labels: the scoring itself is exact integer work;
  * every launch form, several frames per call, open and closed sweeps,
    sub-sampling, segment removal and radii 0 .. 8.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_02704_amd as lp
    c = lp.LidarContext(0)
    yield c
    c.close()


def _oracle_counts(f, s, wrap, labels, R):
    sen = f.sensor
    return oracle.frame_edge_scores(f.xyz, f.prim, sen.n_rings, sen.n_azimuth, s, sen.elevations(), labels,
                                    az0=sen.az0, wrap=wrap, radius=R)


@pytest.mark.parametrize("name,s,wrap,R", [("c1_16x1800", 1, 1, 1), ("c1_16x1800", 1, 0, 0),
                                           ("paper_32x1800", 5, 1, 1), ("paper_32x1800", 15, 1, 2),
                                           ("c2_64x2048", 2, 0, 3), ("c4_128x4096", 2, 1, 8)])
def test_scores_on_oracle_normals(ctx, name, s, wrap, R):
    f = synth.workload_frames(name)[0]
    print(f"case {name} s={s} wrap={wrap} R={R} N={f.n_points}", flush=True)
    r = run_oracle(f.xyz, f.sensor, s, wrap)
    g = run_gpu(ctx, [(f.xyz, f.sensor, s, wrap, r.normals, f.prim)], score_radius=R)[0]
    assert np.array_equal(g["labels"], r.labels)
    want = _oracle_counts(f, s, wrap, r.labels, R)
    assert want[0] > 0 and want[1] > 0
    assert g["edge_counts"] == want


@pytest.mark.parametrize("name,s", [("c2_64x2048", 1), ("c4_128x4096", 2)])
def test_scores_of_gpu_labels_on_raw_sweeps(ctx, name, s):
    f = synth.workload_frames(name)[0]
    for R in (0, 1, 4):
        g = run_gpu(ctx, [(f.xyz, f.sensor, s, 1, None, f.prim)], score_radius=R)[0]
        assert g["edge_counts"] == _oracle_counts(f, s, 1, g["labels"], R), R


def test_scores_with_segment_removal(ctx):
    f = synth.workload_frames("paper_32x1800")[0]
    r = run_oracle(f.xyz, f.sensor, 5, min_segment=4)
    g = run_gpu(ctx, [(f.xyz, f.sensor, 5, 1, r.normals, f.prim)], min_segment=4, score_radius=1)[0]
    assert np.array_equal(g["labels"], r.labels)
    assert g["edge_counts"] == _oracle_counts(f, 5, 1, r.labels, 1)


def test_scores_in_every_launch_form(ctx):
    frames = synth.batch_frames(6, 99)
    refs = [run_oracle(f.xyz, f.sensor, 1) for f in frames]
    want = [_oracle_counts(f, 1, 1, r.labels, 2) for f, r in zip(frames, refs)]
    items = [(f.xyz, f.sensor, 1, 1, r.normals, f.prim) for f, r in zip(frames, refs)]
    for launch in ("plain", "batched", "graph", "graph"):
        got = run_gpu(ctx, items, launch=launch, score_radius=2)
        for k, (g, w) in enumerate(zip(got, want)):
            assert g["edge_counts"] == w, (launch, k)
    # a batch where only some frames ask for scores, and then none: the others are untouched
    import torch
    import paper_2005_02704_amd as lp
    from gpu_helpers import geometry, pad_normals
    inputs = [(torch.from_numpy(f.xyz).cuda(), geometry(f.sensor), torch.from_numpy(pad_normals(r.normals, f.sensor)).cuda(),
               torch.from_numpy(f.prim.astype(np.int32)).cuda()) for f, r in zip(frames, refs)]
    outs = [lp.Outputs(geometry(f.sensor), torch.device("cuda", 0), scores=(k % 2 == 0)) for k, f in enumerate(frames)]
    prep = ctx.prepare(inputs, lp.make_params(score_radius=2), outs)
    for launch in ("batched", "graph"):
        ctx.lidar_mesh_segment(prep, launch=launch)
        torch.cuda.synchronize()
        for k, o in enumerate(outs):
            if k % 2 == 0:
                assert tuple(int(x) for x in o.edge_counts.cpu()) == want[k], (launch, k)
            else:
                assert o.edge_counts is None


def test_score_arguments_rejected(ctx):
    import torch
    import paper_2005_02704_amd as lp
    from gpu_helpers import geometry
    f = synth.workload_frames("c1_16x1800")[0]
    x = torch.from_numpy(f.xyz).cuda()
    out = lp.Outputs(geometry(f.sensor), torch.device("cuda", 0), scores=True)
    with pytest.raises(lp.LidarError):   # no truth ids
        ctx.lidar_mesh_segment(ctx.prepare([(x, geometry(f.sensor), None)], lp.make_params(), [out]))
    tr = torch.from_numpy(f.prim.astype(np.int32)).cuda()
    with pytest.raises(lp.LidarError):   # radius beyond the maximum
        ctx.lidar_mesh_segment(ctx.prepare([(x, geometry(f.sensor), None, tr)],
                                           lp.make_params(score_radius=lp.LIDAR_MAX_SCORE_RADIUS + 1), [out]))
