"""The C-ABI library loads and exports every symbol include/lidarseg.h declares
(no device calls: these run on the CPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lidarseg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lidar_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2005_02704_amd as lp
    L = lp.load_library()
    declared = _declared()
    assert set(declared) == set(lp.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_query_sizes_and_validation_on_host():
    import paper_2005_02704_amd as lp
    geo = lp.SensorGeometry(np.radians(np.linspace(15, -15, 16)), 1800, 1)
    assert lp.lidar_query_sizes(geo) == (16 * 1800, 2 * 15 * 1800)
    geo = lp.SensorGeometry(np.radians(np.linspace(15, -15, 16)), 1800, 7)   # 7 does not divide 1800
    with pytest.raises(lp.LidarError):
        lp.lidar_query_sizes(geo)
    geo = lp.SensorGeometry(np.radians(np.linspace(-15, 15, 16)), 1800, 1)   # ascending
    with pytest.raises(lp.LidarError):
        lp.lidar_query_sizes(geo)
    geo = lp.SensorGeometry(np.radians(np.linspace(15, -15, 200)), 1800, 1)  # too many rings
    with pytest.raises(lp.LidarError):
        lp.lidar_query_sizes(geo)
    geo = lp.SensorGeometry(np.radians(np.linspace(15, -15, 16)), 2, 1, wrap=1)
    with pytest.raises(lp.LidarError):
        lp.lidar_query_sizes(geo)
