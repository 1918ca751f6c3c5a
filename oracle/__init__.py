"""FP64 CPU oracle of the hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it.

The arithmetic lives in ``lidar_oracle.c`` (plain C, FP64); this module builds
it with gcc and marshals numpy arrays through ctypes.  Grids use the firing
order layout: cell (ring i, sampled column k) at index k*H + i.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lidar_oracle.c")
_LIB = os.path.join(_HERE, "liblidar_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, so FP64 follows the source order)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.oracle_bin.argtypes = [P, i64, i32, i32, i32, P, f64, f64, f64, P]
        L.oracle_bin.restype = i64
        L.oracle_vertex_index.argtypes = [i32, i32, P, P]
        L.oracle_vertex_index.restype = i64
        L.oracle_mesh_mask.argtypes = [i32, i32, i32, P, P]
        L.oracle_mesh_mask.restype = None
        L.oracle_triangles.argtypes = [i32, i32, i32, P, P]
        L.oracle_triangles.restype = i64
        L.oracle_normals.argtypes = [i32, i32, i32, P, P, P, P]
        L.oracle_normals.restype = i64
        L.oracle_labels.argtypes = [i32, i32, i32, P, P, P, P, P]
        L.oracle_labels.restype = i64
        L.oracle_mesh_segment.argtypes = [P, i64, i32, i32, i32, i32, P, f64, f64, f64, P,
                                          P, P, P, P, P, P, P]
        L.oracle_mesh_segment.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# stage functions


def bin_points(xyz, H, W, s, elev, az0=0.0, r_min=1.0, r_max=60.0):
    """Steps 1-2: cell_point[k*H+i] = kept point index or -1."""
    xyz = _c(xyz, np.float32).reshape(-1, 3)
    elev = _c(elev, np.float64)
    Wp = W // s
    out = np.empty(H * Wp, dtype=np.int64)
    lib().oracle_bin(_p(xyz), xyz.shape[0], H, W, s, _p(elev), az0, r_min, r_max, _p(out))
    return out


def mesh_mask(H, Wp, wrap, valid):
    valid = _c(valid, np.uint8)
    out = np.empty(H * Wp, dtype=np.uint8)
    lib().oracle_mesh_mask(H, Wp, wrap, _p(valid), _p(out))
    return out


def triangles(H, Wp, wrap, valid):
    valid = _c(valid, np.uint8)
    T = lib().oracle_triangles(H, Wp, wrap, _p(valid), None)
    out = np.empty((max(T, 1), 3), dtype=np.int32)
    lib().oracle_triangles(H, Wp, wrap, _p(valid), _p(out))
    return out[:T]


def normals(H, Wp, wrap, cell_xyz, valid):
    """Step 4 on a grid: returns (normals float64 [cells,3], has_normal uint8 [cells])."""
    cell_xyz = _c(cell_xyz, np.float32).reshape(-1, 3)
    valid = _c(valid, np.uint8)
    n = np.empty((H * Wp, 3), dtype=np.float64)
    h = np.empty(H * Wp, dtype=np.uint8)
    lib().oracle_normals(H, Wp, wrap, _p(cell_xyz), _p(valid), _p(n), _p(h))
    return n, h


def labels(H, Wp, wrap, valid, has_normal, normals32, thr=(0.2, 0.2, 0.2)):
    """Step 5 (Algorithm 1) on a grid: labels per cell (0 = empty cell), K."""
    valid = _c(valid, np.uint8)
    has_normal = _c(has_normal, np.uint8)
    normals32 = _c(normals32, np.float32).reshape(-1, 3)
    thr = _c(thr, np.float64)
    out = np.empty(H * Wp, dtype=np.int32)
    K = lib().oracle_labels(H, Wp, wrap, _p(valid), _p(has_normal), _p(normals32), _p(thr), _p(out))
    return out, int(K)


@dataclass
class Result:
    vertices: np.ndarray      # float32 [V,3]
    normals: np.ndarray       # float32 [V,3]
    labels: np.ndarray        # int32 [V]
    triangles: np.ndarray     # int32 [T,3]
    vertex_point: np.ndarray  # int32 [V]
    normals64: np.ndarray     # float64 [V,3]

    @property
    def counts(self):
        return (self.vertices.shape[0], self.triangles.shape[0],
                int(self.labels.max()) if self.labels.size else 0)


def mesh_segment(xyz, H, W, s, elev, *, az0=0.0, r_min=1.0, r_max=60.0, thr=(0.2, 0.2, 0.2),
                 wrap=1) -> Result:
    """The whole path on one sweep (compact outputs in vertex order)."""
    xyz = _c(xyz, np.float32).reshape(-1, 3)
    elev = _c(elev, np.float64)
    thr = _c(thr, np.float64)
    Wp = W // s
    cells = H * Wp
    V = np.empty((cells, 3), np.float32)
    Nn = np.empty((cells, 3), np.float32)
    L = np.empty(cells, np.int32)
    T = np.empty((2 * cells + 1, 3), np.int32)
    VP = np.empty(cells, np.int32)
    N64 = np.empty((cells, 3), np.float64)
    cnt = np.zeros(3, np.int64)
    rc = lib().oracle_mesh_segment(_p(xyz), xyz.shape[0], H, W, s, wrap, _p(elev), az0, r_min, r_max,
                                   _p(thr), _p(V), _p(Nn), _p(L), _p(T), _p(VP), _p(cnt), _p(N64))
    if rc != 0:
        raise ValueError("oracle_mesh_segment: bad arguments")
    v, t = int(cnt[0]), int(cnt[1])
    return Result(V[:v].copy(), Nn[:v].copy(), L[:v].copy(), T[:t].copy(), VP[:v].copy(), N64[:v].copy())


def mesh_segment_frame(frame, s=1, **kw) -> Result:
    """Convenience: run on a synth.Frame."""
    sen = frame.sensor
    return mesh_segment(frame.xyz, sen.n_rings, sen.n_azimuth, s, sen.elevations(), az0=sen.az0, **kw)
