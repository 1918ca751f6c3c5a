"""The no-allocation entry point, lidar_mesh_segment_noalloc, against
lidar_mesh_segment on the same inputs: the same outputs bit for bit (counts,
vertices, normals, labels, triangles, vertex_point, point labels), on two calls
in a row whose second input is smaller, in the plain and batched forms; its
refusals (graph form, too many frames, a batch above the scratch size), made
before anything is enqueued; and that the context's own workspace is never
allocated by it."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _prepare(ctx, frames, subs, dev, params, point_labels=False):
    import torch
    import paper_2005_02704_amd as lp
    geos = [lp.SensorGeometry(f.sensor.elevations(), f.sensor.n_azimuth, s, 1, f.sensor.az0)
            for f, s in zip(frames, subs)]
    outs = [lp.Outputs(g, dev, n_points=f.xyz.shape[0] if point_labels else 0) for f, g in zip(frames, geos)]
    for o in outs:   # every output the call must write starts as garbage
        for t in (o.vertices, o.normals, o.labels, o.triangles, o.vertex_point, o.counts, o.point_labels):
            if t is not None:
                t.fill_(-7)
    inputs = [(torch.from_numpy(f.xyz).to(dev), g, None) for f, g in zip(frames, geos)]
    return ctx.prepare(inputs, params, outs), outs


def _snap(outs):
    snaps = []
    for o in outs:
        c = o.counts.cpu()
        V, T = int(c[0]), int(c[1])
        assert V >= 0 and T >= 0 and int(c[2]) >= 0
        snaps.append(dict(counts=c.numpy(), vertices=o.vertices[:V].cpu().numpy(),
                          normals=o.normals[:V].cpu().numpy(), labels=o.labels[:V].cpu().numpy(),
                          triangles=o.triangles[:T].cpu().numpy(), vertex_point=o.vertex_point[:V].cpu().numpy(),
                          point_labels=o.point_labels.cpu().numpy() if o.point_labels is not None else None))
    return snaps


def _assert_same(got, want):
    assert len(got) == len(want)
    for f, (g, w) in enumerate(zip(got, want)):
        for k in w:
            if w[k] is None:
                assert g[k] is None
                continue
            # normals compared as bits: the same kernels on the same inputs
            a, b = (g[k].view(np.uint32), w[k].view(np.uint32)) if k == "normals" else (g[k], w[k])
            assert np.array_equal(a, b), (f, k)


def _both(frames, subs, dev, launch, params, point_labels=False, na_ctx=None):
    """Outputs of the no-allocation entry point (on na_ctx) and of
    lidar_mesh_segment (on a context of its own) for the same inputs."""
    import torch
    import paper_2005_02704_amd as lp
    ref_ctx = lp.LidarContext(0)
    try:
        pr, orf = _prepare(ref_ctx, frames, subs, dev, params, point_labels)
        ref_ctx.lidar_mesh_segment(pr, launch=launch)
        pn, ona = _prepare(na_ctx, frames, subs, dev, params, point_labels)
        na_ctx.lidar_mesh_segment_noalloc(pn, launch=launch)
        torch.cuda.synchronize()
        return _snap(ona), _snap(orf)
    finally:
        ref_ctx.close()


@pytest.mark.parametrize("launch", ["batched", "plain"])
def test_noalloc_equals_the_allocating_entry_point(dev, launch):
    import paper_2005_02704_amd as lp
    params = lp.make_params()
    ctx = lp.LidarContext(0)
    try:
        first = synth.batch_frames(6, 7)                       # uneven sweeps, up to 128 x 4096
        second = [synth.workload_frames("c1_16x1800")[0]]      # one small sweep
        print(f"{launch}: first call {len(first)} sweeps, "
              f"{sum(f.sensor.n_rings * f.sensor.n_azimuth for f in first)} cells", flush=True)
        got, want = _both(first, [1] * len(first), dev, launch, params, na_ctx=ctx)
        _assert_same(got, want)
        print(f"{launch}: second call, 1 sweep of 16 x 1800", flush=True)
        got, want = _both(second, [1], dev, launch, params, na_ctx=ctx)
        _assert_same(got, want)
        assert ctx.workspace_bytes() == 0   # the context allocated no workspace of its own
    finally:
        ctx.close()


def test_noalloc_point_labels_and_segment_removal(dev):
    import paper_2005_02704_amd as lp
    params = lp.make_params(min_segment=3)
    ctx = lp.LidarContext(0)
    try:
        big = synth.workload_frames("c2_64x2048")[0]
        small = synth.workload_frames("c1_16x1800")[0]
        print("point labels, s = 2, 64 x 2048, then 16 x 1800", flush=True)
        for frames, subs in (([big, small], [2, 1]), ([small], [1])):
            got, want = _both(frames, subs, dev, "batched", params, point_labels=True, na_ctx=ctx)
            _assert_same(got, want)
        assert ctx.workspace_bytes() == 0
    finally:
        ctx.close()


def test_noalloc_refusals_enqueue_nothing(dev):
    import torch
    import paper_2005_02704_amd as lp
    params = lp.make_params()
    ctx = lp.LidarContext(0)
    try:
        small = synth.workload_frames("c1_16x1800")[0]
        p, outs = _prepare(ctx, [small], [1], dev, params)
        with pytest.raises(lp.LidarError) as err:
            ctx.lidar_mesh_segment_noalloc(p, launch="graph")
        assert err.value.code == lp.LIDAR_EINVAL
        p, outs = _prepare(ctx, [small] * (lp.LIDAR_NOALLOC_MAX_FRAMES + 1),
                           [1] * (lp.LIDAR_NOALLOC_MAX_FRAMES + 1), dev, params)
        with pytest.raises(lp.LidarError) as err:
            ctx.lidar_mesh_segment_noalloc(p, launch="batched")
        assert err.value.code == lp.LIDAR_EINVAL
        # 128 x 65536 cells need about 100 MB of workspace: above the scratch
        g = lp.SensorGeometry(np.radians(np.linspace(15.0, -25.0, 128)), 65536, 1)
        xyz = torch.tensor([[10.0, 0.0, 0.0]], dtype=torch.float32, device=dev)
        o = lp.Outputs(g, dev)
        o.counts.fill_(-7)
        p = ctx.prepare([(xyz, g, None)], params, [o])
        with pytest.raises(lp.LidarError) as err:
            ctx.lidar_mesh_segment_noalloc(p, launch="batched")
        assert err.value.code == lp.LIDAR_ENOMEM
        assert "bytes" in str(err.value)
        torch.cuda.synchronize()
        assert o.counts.cpu().tolist() == [-7, -7, -7]   # nothing ran
        assert ctx.workspace_bytes() == 0
        del o, p
    finally:
        ctx.close()
