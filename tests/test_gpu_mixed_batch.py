"""One batched call whose frames differ in every per-frame option: sampling
interval, open or closed seam, caller-given normals or computed ones, every
input point's label asked for or not.  Each frame's outputs equal (bit for bit)
the same frame called alone, in the batched and the graph forms, and the
alone calls match the oracle."""
import numpy as np
import pytest

import synth
from gpu_helpers import THR, check_geometry, geometry, pad_normals, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

# (workload, s, wrap, give the oracle's normals, ask for point labels)
MIX = [("c1_16x1800", 1, 1, False, True),
       ("c2_64x2048", 2, 0, True, False),
       ("paper_32x1800", 5, 1, False, True),
       ("c2_64x2048", 4, 1, False, False),
       ("c4_128x4096", 2, 0, True, True)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_02704_amd as lp
    c = lp.LidarContext(0)
    yield c
    c.close()


def test_mixed_options_in_one_batch(ctx):
    import torch
    import paper_2005_02704_amd as lp
    frames, alone, inputs, outs = [], [], [], []
    dev = torch.device("cuda", 0)
    for name, s, wrap, give_normals, want_points in MIX:
        f = synth.workload_frames(name)[0]
        ref = run_oracle(f.xyz, f.sensor, s, wrap, point_labels=want_points)
        nin = ref.normals if give_normals else None
        a = run_gpu(ctx, [(f.xyz, f.sensor, s, wrap, nin)], launch="plain", point_labels=want_points)[0]
        check_geometry(a, ref)
        if give_normals:
            # labels on the oracle's own normals are the oracle's labels
            assert np.array_equal(a["labels"], ref.labels), name
            if want_points:
                assert np.array_equal(a["point_labels"], ref.point_labels), name
        if want_points:
            assert a["point_labels"] is not None and a["point_labels"].shape[0] == f.n_points
        frames.append((name, s, wrap, give_normals, want_points))
        alone.append(a)
        g = geometry(f.sensor, s, wrap)
        x = torch.from_numpy(np.ascontiguousarray(f.xyz, np.float32)).to(dev)
        n = torch.from_numpy(pad_normals(nin, f.sensor, s)).to(dev) if give_normals else None
        inputs.append((x, g, n))
        outs.append(lp.Outputs(g, dev, n_points=f.n_points if want_points else 0))
    print(f"mixed batch of {len(MIX)} frames", flush=True)
    params = lp.make_params(1.0, 60.0, THR)
    prep = ctx.prepare(inputs, params, outs)
    stream = torch.cuda.current_stream(dev)
    for launch in ("batched", "graph"):
        torch.cuda.synchronize()
        ctx.lidar_mesh_segment(prep, stream, launch)
        torch.cuda.synchronize()
        for (name, s, wrap, give_normals, want_points), o, a in zip(frames, outs, alone):
            t = o.trimmed()
            tag = (launch, name, s, wrap, give_normals, want_points)
            assert t["counts"] == a["counts"], tag
            for key in ("vertices", "labels", "triangles", "vertex_point"):
                assert np.array_equal(t[key].cpu().numpy(), a[key]), (tag, key)
            assert np.array_equal(t["normals"].cpu().numpy().view(np.uint32), a["normals"].view(np.uint32)), tag
            if want_points:
                assert np.array_equal(t["point_labels"].cpu().numpy(), a["point_labels"]), tag
            else:
                assert t["point_labels"] is None
