"""Normals on grazing ground, where the mesh triangles are thinnest.

Far rings meet the ground at grazing angles, so the triangles there are long
and thin.  A normal computed from inexact edge vectors is then least accurate:
its direction error grows like the rounding error over the sine of the
triangle's smallest angle.  The sweeps here are ground alone (tilted 0-8
degrees, so the points do not lie on a float plane), at 16, 32, 64 and 128
rings, 1800 and 4096 firings (the x and y axis crossings included), without
and with range noise.  The GPU normals must lie within 5e-6 rad of the
oracle's FP64 normals, half the parity bar, and the has-normal sets must
agree exactly."""
import numpy as np
import pytest

import synth
from gpu_helpers import normal_angles, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

GRAZING_TOL_RAD = 5e-6


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_02704_amd as lp
    c = lp.LidarContext(0)
    yield c
    c.close()


@pytest.mark.parametrize("H", [16, 32, 64, 128])
@pytest.mark.parametrize("W", [1800, 4096])
@pytest.mark.parametrize("sigma", [0.0, 0.01])
def test_grazing_ground_normals(ctx, H, W, sigma):
    sensor = synth.Sensor.standard(H, W)
    worst = 0.0
    for seed in (11, 12):
        f = synth.make_frame(sensor, "sloped_ground", seed, sigma=sigma, dropout=0.0)
        g = run_gpu(ctx, [(f.xyz, sensor, 1, 1, None)])[0]
        r = run_oracle(f.xyz, sensor)
        assert g["counts"][0] == r.vertices.shape[0]
        hg = np.any(g["normals"] != 0, axis=1)
        hr = np.any(r.normals64 != 0, axis=1)
        assert np.array_equal(hg, hr)
        ang = normal_angles(g["normals"][hg], r.normals64[hr])
        worst = max(worst, float(ang.max()) if ang.size else 0.0)
    print(f"H={H} W={W} sigma={sigma}: largest angle {worst:.2e} rad", flush=True)
    assert worst <= GRAZING_TOL_RAD
