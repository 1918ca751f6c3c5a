"""GPU edge cases against the oracle: empty and degenerate sweeps, seams, ragged tiles."""
import math

import numpy as np
import pytest

import synth
from gpu_helpers import check_geometry, run_gpu, run_oracle

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


def _both(ctx, xyz, sen, s=1, wrap=1, **kw):
    g = run_gpu(ctx, [(xyz, sen, s, wrap, None)], **kw)[0]
    r = run_oracle(xyz, sen, s, wrap, **kw)
    check_geometry(g, r)
    assert g["counts"][2] == r.counts[2]
    assert np.array_equal(g["labels"], r.labels)
    return g, r


def test_empty_sweep(ctx):
    sen = synth.Sensor.standard(16, 1024)
    g, r = _both(ctx, np.zeros((0, 3), np.float32), sen)
    assert g["counts"] == (0, 0, 0)


def test_all_points_out_of_range(ctx):
    f = synth.workload_frames("c1_16x1800")[0]
    g, _ = _both(ctx, f.xyz, f.sensor, r_min=500.0, r_max=600.0)
    assert g["counts"] == (0, 0, 0)


def test_single_point(ctx):
    sen = synth.Sensor.standard(16, 1024)
    g, _ = _both(ctx, np.array([[10.0, 0.0, -0.5]], np.float32), sen)
    assert g["counts"] == (1, 0, 1)


def test_single_ring(ctx):
    sen = synth.Sensor(1, 720, 0.0, 0.0)
    ang = np.arange(720) * 2 * math.pi / 720
    xyz = np.stack([10 * np.cos(ang), 10 * np.sin(ang), np.zeros(720)], 1).astype(np.float32)
    g, _ = _both(ctx, xyz, sen)
    assert g["counts"] == (720, 0, 720)
    assert not np.any(g["normals"])


@pytest.mark.parametrize("W,s,wrap", [(3, 1, 1), (4, 1, 1), (6, 2, 1), (5, 1, 0), (1, 1, 0), (2, 1, 0)])
def test_tiny_lattices(ctx, W, s, wrap):
    sen = synth.Sensor(5, W, 10.0, -10.0)
    rng = np.random.Generator(np.random.PCG64(W * 10 + s))
    U = sen.rays().transpose(1, 0, 2).reshape(-1, 3)
    r = rng.uniform(5, 6, size=U.shape[0])
    keep = rng.random(U.shape[0]) < 0.85
    xyz = (U * r[:, None])[keep].astype(np.float32)
    _both(ctx, xyz, sen, s, wrap)


@pytest.mark.parametrize("H,W", [(7, 1000), (128, 1800), (100, 333), (33, 4097), (16, 1800)])
def test_ragged_tiles_and_odd_ring_counts(ctx, H, W):
    sen = synth.Sensor(H, W, 12.0, -24.0)
    f = synth.make_frame(sen, "street", H * 7 + W, sigma=0.01, dropout=0.2)
    g = run_gpu(ctx, [(f.xyz, sen, 1, 1, None)])[0]
    r = run_oracle(f.xyz, sen, 1, 1)
    check_geometry(g, r)
    nin_g = run_gpu(ctx, [(f.xyz, sen, 1, 1, r.normals)])[0]
    assert np.array_equal(nin_g["labels"], r.labels)


def test_widest_sweep_at_the_most_rings(ctx):
    """One sweep of 128 rings x 65 536 firings (8.4 M cells, 4 096 tiles of 2 048
    cells, one frame): index arithmetic past 2^24 points and cells, the longest
    sums over earlier tiles, in the batched and graph forms and at the largest
    tile shape.  Geometry against the oracle, labels bit-exact on the oracle's
    normals, and the labels of the GPU's own normals between the oracle's
    thr -/+ 1e-4 partitions."""
    from gpu_helpers import sandwich
    sen = synth.Sensor.standard(128, 65536)
    f = synth.make_frame(sen, "street", 5, sigma=0.01, dropout=0.1)
    print(f"widest sweep: {f.n_points} points", flush=True)
    r = run_oracle(f.xyz, sen, 1, 1)
    ctx.set_tuning(0, 2048, 512)
    try:
        g = run_gpu(ctx, [(f.xyz, sen, 1, 1, None)], launch="graph")[0]
        check_geometry(g, r)
        assert sandwich(g["labels"], f.xyz, sen, 1)
        on_ref = run_gpu(ctx, [(f.xyz, sen, 1, 1, r.normals)], launch="batched")[0]
        assert on_ref["counts"] == tuple(int(v) for v in r.counts)
        assert np.array_equal(on_ref["labels"], r.labels)
    finally:
        ctx.set_tuning(0, 0, 0)


def test_open_sweep_without_seam(ctx):
    f = synth.workload_frames("c2_64x2048")[0]
    r = run_oracle(f.xyz, f.sensor, 2, 0)
    g = run_gpu(ctx, [(f.xyz, f.sensor, 2, 0, r.normals)])[0]
    check_geometry(g, r)
    assert np.array_equal(g["labels"], r.labels)


def test_non_finite_and_duplicate_points(ctx):
    f = synth.workload_frames("c1_16x1800")[0]
    xyz = f.xyz.copy()
    xyz[3, 0] = np.nan
    xyz[50, 2] = np.inf
    dup = np.concatenate([xyz, xyz[::7], xyz[::5] * np.float32(1.0001)])
    _both(ctx, dup, f.sensor)


def test_noise_free_ground_normals_bitwise(ctx):
    sen = synth.Sensor.standard(32, 1024)
    f = synth.make_frame(sen, "ground", 2, sigma=0.0, dropout=0.0)
    g, r = _both(ctx, f.xyz, sen)
    has = np.any(g["normals"] != 0, axis=1)
    assert np.all(g["normals"][has] == np.float32([0, 0, -1]))
    assert np.array_equal(g["normals"], r.normals)


def test_repeat_runs_bitwise(ctx):
    f = synth.workload_frames("c4_128x4096")[0]
    a = run_gpu(ctx, [(f.xyz, f.sensor, 2, 1, None)], launch="batched")[0]
    for _ in range(3):
        b = run_gpu(ctx, [(f.xyz, f.sensor, 2, 1, None)], launch="batched")[0]
        for k in ("vertices", "normals", "labels", "triangles", "vertex_point"):
            assert np.array_equal(a[k], b[k])


def test_reported_rings(ctx):
    """Rings the sensor reports replace the elevation decision: equal to the
    generating rings they change nothing; relabelled (and some out of range)
    they move the points exactly as in the oracle."""
    f = synth.workload_frames("c2_64x2048")[0]
    sen = f.sensor
    H = sen.n_rings
    plain = run_gpu(ctx, [(f.xyz, sen, 2, 1, None)], launch="batched")[0]
    same = run_gpu(ctx, [(f.xyz, sen, 2, 1, None, None, f.ring.astype(np.uint8))], launch="batched")[0]
    for k in ("vertices", "normals", "labels", "triangles", "vertex_point"):
        assert np.array_equal(plain[k], same[k]), k
    rng = np.random.Generator(np.random.PCG64(9))
    reported = rng.permutation(H)[f.ring].astype(np.uint8)
    reported[rng.random(f.n_points) < 0.03] = 200
    r = run_oracle(f.xyz, sen, 2, ring_ids=reported, point_labels=True)
    for launch in ("plain", "graph"):
        g = run_gpu(ctx, [(f.xyz, sen, 2, 1, None, None, reported)], launch=launch, point_labels=True)[0]
        check_geometry(g, r)
        g2 = run_gpu(ctx, [(f.xyz, sen, 2, 1, r.normals, None, reported)], launch=launch, point_labels=True)[0]
        assert np.array_equal(g2["labels"], r.labels)
        assert np.array_equal(g2["point_labels"], r.point_labels)


def test_call_arguments_are_rejected_before_any_work(ctx):
    """Every bad argument of lidar_mesh_segment returns LIDAR_EINVAL with a
    message, and the context stays usable."""
    import ctypes
    import torch
    import paper_2005_02704_amd as lp
    from paper_2005_02704_amd import lidarseg as b
    from gpu_helpers import geometry
    f = synth.workload_frames("c1_16x1800")[0]
    geo = geometry(f.sensor)
    x = torch.from_numpy(f.xyz).cuda()
    dev = torch.device("cuda", 0)

    def call(params=None, launch="batched", outs=None, inputs=None):
        o = outs or [lp.Outputs(geo, dev)]
        prep = ctx.prepare(inputs or [(x, geo, None)], params or lp.make_params(), o)
        ctx.lidar_mesh_segment(prep, launch=launch)

    bad_params = [lp.make_params(r_min=-1.0), lp.make_params(r_min=5.0, r_max=4.0),
                  lp.make_params(r_max=float("inf")), lp.make_params(thr=(0.2, 0.0, 0.2)),
                  lp.make_params(thr=(0.2, 0.2, float("nan"))), lp.make_params(predicate=7),
                  lp.make_params(predicate=lp.LIDAR_PRED_COSINE, cos_min=1.0), lp.make_params(min_segment=-2)]
    for p in bad_params:
        with pytest.raises(lp.LidarError) as e:
            call(params=p)
        assert e.value.code == lp.LIDAR_EINVAL and str(e.value)
    with pytest.raises(lp.LidarError):
        call(launch=9)
    # a required output missing
    o = lp.Outputs(geo, dev)
    prep = ctx.prepare([(x, geo, None)], lp.make_params(), [o])
    prep[3][0].labels = None
    with pytest.raises(lp.LidarError):
        ctx.lidar_mesh_segment(prep)
    # points given without coordinates
    prep = ctx.prepare([(x, geo, None)], lp.make_params(), [lp.Outputs(geo, dev)])
    prep[0][0].xyz = None
    with pytest.raises(lp.LidarError):
        ctx.lidar_mesh_segment(prep)
    # a sensor the library refuses (elevations ascending)
    bad_geo = lp.SensorGeometry(f.sensor.elevations()[::-1].copy(), f.sensor.n_azimuth, 1)
    with pytest.raises(lp.LidarError):
        call(inputs=[(x, bad_geo, None)], outs=[lp.Outputs(geo, dev)])
    # tuning arguments
    for args in ((-1, 0, 0), (0, 768, 256), (0, 512, 512)):
        with pytest.raises(lp.LidarError):
            ctx.set_tuning(*args)
    for stage, wg in ((-1, 4), (lp.LIDAR_N_STAGES, 4), (0, -3)):
        with pytest.raises(lp.LidarError):
            ctx.set_stage_grid(stage, wg)
    # and the context still works
    g = run_gpu(ctx, [(f.xyz, f.sensor, 1, 1, None)], launch="batched")[0]
    r = run_oracle(f.xyz, f.sensor, 1)
    check_geometry(g, r)
