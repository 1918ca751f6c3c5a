"""Served form on the GPU: a Poisson mix from several sensors through the
continuous-batching server; every result equals the same sweep run alone."""
import numpy as np
import pytest

import synth
from paper_2005_02704_amd.serve import GpuExecutor, Request, Server, poisson_schedule

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("launch,max_batch", [("graph", 8), ("batched", 8), ("plain", 1)])
def test_served_mix_equals_alone(launch, max_batch):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_02704_amd as lp
    sensors = [s for s, _ in synth.served_sensors(8)][:5]
    pool = [[synth.make_frame(s, "street", 500 + 10 * q + k, sigma=0.01, dropout=0.1) for k in range(2)]
            for q, s in enumerate(sensors)]
    geos = [lp.SensorGeometry(s.elevations(), s.n_azimuth, 1, 1, s.az0) for s in sensors]
    pinned = [[torch.from_numpy(f.xyz).pin_memory() for f in row] for row in pool]

    ex = GpuExecutor(geos, n_slots=3, launch=launch, copy_mesh=True)
    srv = Server(ex, budget_bytes=1 << 30, max_batch=max_batch)

    def make(rid, s, k, t):
        return Request(rid, s, pinned[s][k], pool[s][k].n_points, t)

    sched = poisson_schedule([400.0] * len(sensors), 0.25, seed=5, n_payloads=2)
    print(f"serving {len(sched)} requests", flush=True)
    wall = srv.run_schedule(sched, make)
    st = srv.stats(wall)
    print(st, flush=True)
    assert st["requests"] == len(sched)
    if max_batch > 1:
        assert st["max_slots_in_flight"] >= 2 and st["mean_batch"] > 1.0
    else:
        assert st["mean_batch"] == 1.0

    ctx = lp.LidarContext(0)
    alone = {}
    for s in range(len(sensors)):
        for k in range(2):
            x = torch.from_numpy(pool[s][k].xyz).cuda()
            o = lp.lidar_mesh_segment(ctx, [(x, geos[s], None)], launch="plain")[0].trimmed()
            alone[(s, k)] = {key: (v.cpu().numpy() if hasattr(v, "cpu") else v) for key, v in o.items()}
    ctx.close()
    # a sweep with more points than the sensor has rays is refused at submission
    rays = geos[0].n_rings * geos[0].n_azimuth
    with pytest.raises(ValueError):
        srv.submit(Request(10 ** 6, 0, pinned[0][0], rays + 1, 0.0))
    ex.close()
    for r in srv.done:
        k = [id(t) for t in pinned[r.sensor]].index(id(r.xyz))
        ref = alone[(r.sensor, k)]
        res = r.result
        assert res["counts"] == ref["counts"]
        for key in ("labels", "vertex_point", "normals", "vertices", "triangles"):
            assert np.array_equal(res[key], ref[key]), key
