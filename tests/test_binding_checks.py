"""The binding refuses tensors the library could not read or write safely
(wrong device, dtype, layout or size) before anything is launched.  These run
on the CPU: the checks take the device to expect as an argument, so CPU
tensors stand in for device tensors here; the GPU test of the same refusals
through LidarContext.prepare is in test_gpu_entry_points.py."""
import numpy as np
import pytest
import torch

import paper_2005_02704_amd as lp
from paper_2005_02704_amd.lidarseg import check_frame, check_tensor

CPU = torch.device("cpu")


class _Out:
    """Outputs at the capacities of a sensor, on the CPU."""

    def __init__(self, geo, n_points=0, scores=False, labels=True, vertex_point=True):
        V, T = lp.lidar_query_sizes(geo)
        self.vertices = torch.empty((V, 3), dtype=torch.float32)
        self.normals = torch.empty((V, 3), dtype=torch.float32)
        self.labels = torch.empty(V, dtype=torch.int32) if labels else None
        self.triangles = torch.empty((max(T, 1), 3), dtype=torch.int32)
        self.vertex_point = torch.empty(V, dtype=torch.int32) if vertex_point else None
        self.counts = torch.zeros(3, dtype=torch.int64)
        self.point_labels = torch.empty(n_points, dtype=torch.int32) if n_points else None
        self.edge_counts = torch.zeros(4, dtype=torch.int64) if scores else None


def _geo(H=16, W=360, s=1):
    return lp.SensorGeometry(np.radians(np.linspace(15, -15, H)), W, s)


def _refused(fn, *a, **k):
    with pytest.raises(lp.LidarError) as e:
        fn(*a, **k)
    assert e.value.code == lp.LIDAR_EINVAL
    return str(e.value)


def test_a_well_formed_frame_passes():
    geo = _geo()
    V, _ = lp.lidar_query_sizes(geo)
    xyz = torch.zeros((100, 3))
    nin = torch.zeros((V, 3))
    check_frame(CPU, xyz, geo, nin, torch.zeros(100, dtype=torch.int32), torch.zeros(100, dtype=torch.uint8),
                _Out(geo, n_points=100, scores=True))
    check_frame(CPU, torch.zeros((0, 3)), geo, None, None, None, _Out(geo, labels=False, vertex_point=False))


def test_points_refused():
    geo = _geo()
    out = _Out(geo)
    assert "float64" in _refused(check_frame, CPU, torch.zeros((10, 3), dtype=torch.float64), geo, None, None,
                                 None, out)
    assert "contiguous" in _refused(check_frame, CPU, torch.zeros((3, 10)).t(), geo, None, None, None, out)
    assert "shape" in _refused(check_frame, CPU, torch.zeros((10, 4)), geo, None, None, None, out)
    assert "shape" in _refused(check_frame, CPU, torch.zeros(30), geo, None, None, None, out)
    # a host tensor where a device tensor is expected
    assert "not cuda:0" in _refused(check_frame, torch.device("cuda", 0), torch.zeros((10, 3)), geo, None, None,
                                    None, out)


def test_short_or_mistyped_side_inputs_refused():
    geo = _geo()
    V, _ = lp.lidar_query_sizes(geo)
    xyz = torch.zeros((50, 3))
    out = _Out(geo)
    assert "rows" in _refused(check_frame, CPU, xyz, geo, torch.zeros((V - 1, 3)), None, None, out)
    assert "float16" in _refused(check_frame, CPU, xyz, geo, torch.zeros((V, 3), dtype=torch.float16), None,
                                 None, out)
    assert "rows" in _refused(check_frame, CPU, xyz, geo, None, torch.zeros(49, dtype=torch.int32), None, out)
    assert "int64" in _refused(check_frame, CPU, xyz, geo, None, torch.zeros(50, dtype=torch.int64), None, out)
    assert "int32" in _refused(check_frame, CPU, xyz, geo, None, None, torch.zeros(50, dtype=torch.int32), out)


@pytest.mark.parametrize("field,bad", [
    ("vertices", torch.empty((10, 3))),
    ("normals", torch.empty((16 * 360, 3), dtype=torch.float64)),
    ("labels", torch.empty(16 * 360 - 1, dtype=torch.int32)),
    ("triangles", torch.empty((3, 2 * 15 * 360), dtype=torch.int32).t()),
    ("vertex_point", torch.empty(16 * 360, dtype=torch.int64)),
    ("counts", torch.zeros(2, dtype=torch.int64)),
    ("point_labels", torch.empty(99, dtype=torch.int32)),
    ("edge_counts", torch.zeros(4, dtype=torch.int32)),
])
def test_outputs_smaller_than_the_capacities_refused(field, bad):
    geo = _geo()
    out = _Out(geo, n_points=100, scores=True)
    setattr(out, field, bad)
    msg = _refused(check_frame, CPU, torch.zeros((100, 3)), geo, None, None, None, out)
    assert field in msg


def test_required_tensor_missing_refused():
    assert "required" in _refused(check_tensor, "xyz", None, CPU, torch.float32, 0, 3)
