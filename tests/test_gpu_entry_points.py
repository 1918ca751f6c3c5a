"""The stage entry points (lidar_mesh_normals: binning, mesh and normals only;
lidar_label_grid: labels of given normals) and the workspace limit, through the
C ABI, against the oracle and against lidar_mesh_segment."""
import numpy as np
import pytest

import synth
from gpu_helpers import check_geometry, geometry, pad_normals, run_gpu, run_oracle

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


def _mesh_normals(ctx, items, launch, params=None):
    """items: (xyz numpy, synth.Sensor, s, wrap).  Outputs without labels."""
    import torch
    import paper_2005_02704_amd as lp
    dev = torch.device("cuda", 0)
    inputs, outs = [], []
    for xyz, sen, s, wrap in items:
        geo = geometry(sen, s, wrap)
        inputs.append((torch.from_numpy(np.ascontiguousarray(xyz, np.float32)).cuda(), geo, None))
        outs.append(lp.Outputs(geo, dev, with_labels=False))
    prep = ctx.prepare(inputs, params or lp.make_params(), outs)
    ctx.lidar_mesh_normals(prep, launch=launch)
    torch.cuda.synchronize()
    res = []
    for o in outs:
        t = o.trimmed()
        res.append(dict(vertices=t["vertices"].cpu().numpy(), normals=t["normals"].cpu().numpy(),
                        triangles=t["triangles"].cpu().numpy(), vertex_point=t["vertex_point"].cpu().numpy(),
                        counts=t["counts"]))
    return res


def _batch():
    f1 = synth.workload_frames("c1_16x1800")[0]
    f2 = synth.workload_frames("c2_64x2048")[0]
    sen = synth.Sensor(33, 1001, 12.0, -24.0)
    f3 = synth.make_frame(sen, "street", 77, sigma=0.01, dropout=0.2)
    return [(f1.xyz, f1.sensor, 1, 1), (f2.xyz, f2.sensor, 2, 1), (f3.xyz, sen, 1, 0)]


@pytest.mark.parametrize("launch", ["plain", "batched", "graph"])
def test_mesh_normals_match_the_oracle_and_the_full_call(ctx, launch):
    items = _batch()
    g = _mesh_normals(ctx, items, launch)
    full = run_gpu(ctx, [it + (None,) for it in items], launch=launch)
    for (xyz, sen, s, wrap), a, b in zip(items, g, full):
        r = run_oracle(xyz, sen, s, wrap)
        check_geometry(a, r)
        assert a["counts"][2] == 0
        assert a["counts"][:2] == b["counts"][:2]
        for k in ("vertices", "normals", "triangles", "vertex_point"):
            assert np.array_equal(a[k], b[k]), k


def test_mesh_normals_leave_the_key_grid_empty(ctx):
    """A mesh-only call resets the cells it used, so the calls after it (full or
    mesh-only, any form) see clean state."""
    items = _batch()
    for launch in ("graph", "batched", "plain"):
        _mesh_normals(ctx, items, launch)
        full = run_gpu(ctx, [it + (None,) for it in items], launch=launch)
        for (xyz, sen, s, wrap), b in zip(items, full):
            r = run_oracle(xyz, sen, s, wrap)
            check_geometry(b, r)
            assert b["counts"][2] == r.counts[2]
    g = _mesh_normals(ctx, items[1:2], "graph")[0]
    check_geometry(g, run_oracle(*items[1]))


def test_mesh_normals_read_only_the_range_window(ctx):
    import paper_2005_02704_amd as lp
    items = _batch()[:1]
    odd = lp.make_params(thr=(0.0, -1.0, float("nan")), predicate=9, min_segment=-5)
    g = _mesh_normals(ctx, items, "batched", params=odd)[0]
    check_geometry(g, run_oracle(*items[0]))
    near = _mesh_normals(ctx, items, "batched", params=lp.make_params(r_min=2.0, r_max=20.0))[0]
    check_geometry(near, run_oracle(*items[0], r_min=2.0, r_max=20.0))


def test_mesh_normals_refuse_label_outputs(ctx):
    import torch
    import paper_2005_02704_amd as lp
    f = synth.workload_frames("c1_16x1800")[0]
    geo = geometry(f.sensor)
    x = torch.from_numpy(f.xyz).cuda()
    dev = torch.device("cuda", 0)
    nin = torch.zeros((geo.n_rings * geo.n_cols, 3), dtype=torch.float32, device=dev)
    truth = torch.zeros(f.n_points, dtype=torch.int32, device=dev)
    cases = [([(x, geo, nin)], [lp.Outputs(geo, dev)]),
             ([(x, geo, None)], [lp.Outputs(geo, dev, n_points=f.n_points)]),
             ([(x, geo, None, truth)], [lp.Outputs(geo, dev, scores=True)])]
    for inputs, outs in cases:
        prep = ctx.prepare(inputs, lp.make_params(), outs)
        with pytest.raises(lp.LidarError) as e:
            ctx.lidar_mesh_normals(prep)
        assert e.value.code == lp.LIDAR_EINVAL
    # a full call without labels is refused as before
    prep = ctx.prepare([(x, geo, None)], lp.make_params(), [lp.Outputs(geo, dev, with_labels=False)])
    with pytest.raises(lp.LidarError):
        ctx.lidar_mesh_segment(prep)


@pytest.mark.parametrize("launch", ["plain", "batched", "graph"])
def test_label_grid_on_oracle_normals(ctx, launch):
    import torch
    import paper_2005_02704_amd as lp
    items = _batch()
    refs = [run_oracle(xyz, sen, s, wrap) for xyz, sen, s, wrap in items]
    dev = torch.device("cuda", 0)
    inputs, outs = [], []
    for (xyz, sen, s, wrap), r in zip(items, refs):
        geo = geometry(sen, s, wrap)
        inputs.append((torch.from_numpy(xyz).cuda(), geo, torch.from_numpy(pad_normals(r.normals, sen, s)).cuda()))
        outs.append(lp.Outputs(geo, dev))
    prep = ctx.prepare(inputs, lp.make_params(), outs)
    ctx.lidar_label_grid(prep, launch=launch)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        t = o.trimmed()
        assert t["counts"] == tuple(int(v) for v in r.counts)
        assert np.array_equal(t["labels"].cpu().numpy(), r.labels)
        assert np.array_equal(t["normals"].cpu().numpy(), r.normals)
    # without normals it is refused
    prep = ctx.prepare([(inputs[0][0], inputs[0][1], None)], lp.make_params(), [lp.Outputs(inputs[0][1], dev)])
    with pytest.raises(lp.LidarError) as e:
        ctx.lidar_label_grid(prep)
    assert e.value.code == lp.LIDAR_EINVAL


def test_workspace_limit():
    """A fresh context's first call takes exactly what the batch needs; under a
    lower limit the same call fails with LIDAR_ENOMEM before any work, and the
    context stays usable."""
    import torch
    import paper_2005_02704_amd as lp
    items = [it + (None,) for it in _batch()]
    a = lp.LidarContext(0)
    b = lp.LidarContext(0)
    try:
        assert a.workspace_bytes() == 0
        run_gpu(a, items, launch="batched")
        need = a.workspace_bytes()
        assert need > 0
        b.set_workspace_limit(need - 1)
        with pytest.raises(lp.LidarError) as e:
            run_gpu(b, items, launch="batched")
        assert e.value.code == lp.LIDAR_ENOMEM and "limit" in str(e.value)
        assert b.workspace_bytes() == 0
        b.set_workspace_limit(need)
        g = run_gpu(b, items, launch="graph")
        assert b.workspace_bytes() == need
        for (xyz, sen, s, wrap, _), out in zip(items, g):
            r = run_oracle(xyz, sen, s, wrap)
            check_geometry(out, r)
            assert out["counts"][2] == r.counts[2]
        # a smaller batch fits in what is held; a larger one does not
        run_gpu(b, items[:1], launch="batched")
        big = synth.workload_frames("c4_128x4096")[0]
        with pytest.raises(lp.LidarError) as e:
            run_gpu(b, [(big.xyz, big.sensor, 1, 1, None)], launch="batched")
        assert e.value.code == lp.LIDAR_ENOMEM
        b.set_workspace_limit(0)
        out = run_gpu(b, [(big.xyz, big.sensor, 2, 1, None)], launch="batched")[0]
        check_geometry(out, run_oracle(big.xyz, big.sensor, 2, 1))
        torch.cuda.synchronize()
    finally:
        a.close()
        b.close()


def test_stage_times(ctx):
    """Per-stage timing: every stage of a batched call is timed once; a
    mesh-only call times bin, geom and the key reset (flatten) only."""
    import paper_2005_02704_amd as lp
    items = _batch()
    ctx.set_profiling(True)
    try:
        ctx.stage_times()
        run_gpu(ctx, [it + (None,) for it in items], launch="batched")
        full = ctx.stage_times()
        _mesh_normals(ctx, items, "batched")
        mesh = ctx.stage_times()
    finally:
        ctx.set_profiling(False)
    assert tuple(full) == lp.STAGES == tuple(mesh)
    assert all(n == 1 for _, n in full.values())
    for k in ("bin", "geom", "cc", "merge", "compress", "flatten", "scan", "label"):
        assert full[k][0] > 0, k
    for k in ("bin", "geom", "flatten"):
        assert mesh[k][0] > 0, k


def test_calls_on_one_context_alternate_streams(ctx):
    """Calls on one context name different streams without any host wait in
    between: each call first waits (on the device) for the context's previous
    call, since they share its workspace, so every output equals the same call
    made alone; the geometry also matches the oracle."""
    import torch
    import paper_2005_02704_amd as lp
    dev = torch.device("cuda", 0)
    frames_a = synth.batch_frames(24, 31)
    frames_b = [synth.workload_frames("c4_128x4096")[0], synth.workload_frames("c1_16x1800")[0]]
    s_b = (2, 1)

    def prep(frames, subs):
        geos = [lp.SensorGeometry(f.sensor.elevations(), f.sensor.n_azimuth, s, 1, f.sensor.az0)
                for f, s in zip(frames, subs)]
        outs = [lp.Outputs(g, dev) for g in geos]
        return ctx.prepare([(torch.from_numpy(f.xyz).to(dev), g, None) for f, g in zip(frames, geos)],
                           lp.make_params(), outs), outs

    def snap(outs):
        return [(o.counts.cpu().clone(), o.labels.cpu().clone(), o.normals.cpu().clone(),
                 o.triangles.cpu().clone()) for o in outs]

    def same(a, b):
        for (ca, la, na, ta), (cb, lb, nb, tb) in zip(a, b):
            V, T = int(ca[0]), int(ca[1])
            if not (torch.equal(ca, cb) and torch.equal(la[:V], lb[:V]) and torch.equal(na[:V], nb[:V])
                    and torch.equal(ta[:T], tb[:T])):
                return False
        return True

    pa, oa = prep(frames_a, [1] * len(frames_a))
    pb, ob = prep(frames_b, s_b)
    pa2, oa2 = prep(frames_a, [1] * len(frames_a))
    pb2, ob2 = prep(frames_b, s_b)
    # alone, one call at a time
    for launch in ("batched", "graph"):
        ctx.lidar_mesh_segment(pa, launch=launch)
        torch.cuda.synchronize()
        ref_a = snap(oa)
        ctx.lidar_mesh_segment(pb, launch=launch)
        torch.cuda.synchronize()
        ref_b = snap(ob)
        for rep in range(3):
            for o in oa + ob + oa2 + ob2:
                o.labels.fill_(-7)
                o.counts.fill_(-7)
            torch.cuda.synchronize()
            sa, sb = torch.cuda.Stream(dev), torch.cuda.Stream(dev)
            ctx.lidar_mesh_segment(pa, stream=sa, launch=launch)
            ctx.lidar_mesh_segment(pb, stream=sb, launch=launch)
            ctx.lidar_mesh_segment(pa2, stream=sa, launch=launch)
            ctx.lidar_mesh_segment(pb2, stream=sb, launch=launch)
            torch.cuda.synchronize()
            assert same(snap(oa), ref_a) and same(snap(oa2), ref_a), (launch, rep)
            assert same(snap(ob), ref_b) and same(snap(ob2), ref_b), (launch, rep)
    for f, s, o in zip(frames_b, s_b, ob2):
        t = o.trimmed()
        g = dict(vertices=t["vertices"].cpu().numpy(), normals=t["normals"].cpu().numpy(),
                 triangles=t["triangles"].cpu().numpy(), vertex_point=t["vertex_point"].cpu().numpy(),
                 counts=t["counts"])
        check_geometry(g, run_oracle(f.xyz, f.sensor, s))


def test_prepare_refuses_unsafe_tensors(ctx):
    """The binding refuses, before any launch, tensors the kernels would read or
    write out of bounds: host memory, another dtype, a transposed view, normals
    or outputs smaller than the sensor's capacities."""
    import torch
    import paper_2005_02704_amd as lp
    dev = torch.device("cuda", 0)
    f = synth.workload_frames("c1_16x1800")[0]
    geo = geometry(f.sensor)
    V, T = lp.lidar_query_sizes(geo)
    x = torch.from_numpy(f.xyz).to(dev)
    good = lp.Outputs(geo, dev)
    short = lp.Outputs(geo, dev)
    short.normals = short.normals[:V // 2]
    bad_inputs = [
        ([(torch.from_numpy(f.xyz), geo, None)], [good]),                       # host tensor
        ([(x.double(), geo, None)], [good]),                                    # float64
        ([(x.t().contiguous().t(), geo, None)], [good]),                        # transposed view
        ([(x, geo, torch.zeros((V - 1, 3), device=dev))], [good]),              # short normals_in
        ([(x, geo, None)], [short]),                                            # short output
    ]
    for inputs, outs in bad_inputs:
        with pytest.raises(lp.LidarError) as e:
            ctx.prepare(inputs, lp.make_params(), outs)
        assert e.value.code == lp.LIDAR_EINVAL
    # the context still works
    g = run_gpu(ctx, [(f.xyz, f.sensor, 1, 1, None)])[0]
    check_geometry(g, run_oracle(f.xyz, f.sensor))
