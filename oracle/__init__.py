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
        L.oracle_bin.argtypes = [P, P, i64, i32, i32, i32, P, f64, f64, f64, P]
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
        L.oracle_labels_pred.argtypes = [i32, i32, i32, P, P, P, i32, P, f64, P]
        L.oracle_labels_pred.restype = i64
        L.oracle_prune.argtypes = [P, i64, i64, i32]
        L.oracle_prune.restype = None
        L.oracle_point_cells.argtypes = [P, P, i64, i32, i32, P, f64, f64, f64, P, P]
        L.oracle_point_cells.restype = None
        L.oracle_backfill.argtypes = [i64, P, P, i32, i32, i32, i32, P, P]
        L.oracle_backfill.restype = None
        L.oracle_edge_scores.argtypes = [i32, i32, i32, P, P, i32, P]
        L.oracle_edge_scores.restype = None
        L.oracle_mesh_segment_ex.argtypes = [P, P, i64, i32, i32, i32, i32, P, f64, f64, f64, i32, P, f64, i32,
                                             P, P, P, P, P, P, P, P]
        L.oracle_mesh_segment_ex.restype = ctypes.c_int
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


def _rings(ring_ids, n):
    if ring_ids is None:
        return None, None
    r = _c(ring_ids, np.uint8).reshape(-1)
    assert r.shape[0] == n
    return r, _p(r)


def bin_points(xyz, H, W, s, elev, az0=0.0, r_min=1.0, r_max=60.0, ring_ids=None):
    """Steps 1-2: cell_point[k*H+i] = kept point index or -1.  ring_ids: each
    point's reported ring (uint8), or None to decide rings by elevation."""
    xyz = _c(xyz, np.float32).reshape(-1, 3)
    elev = _c(elev, np.float64)
    rk, rp = _rings(ring_ids, xyz.shape[0])
    Wp = W // s
    out = np.empty(H * Wp, dtype=np.int64)
    lib().oracle_bin(_p(xyz), rp, xyz.shape[0], H, W, s, _p(elev), az0, r_min, r_max, _p(out))
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


def labels(H, Wp, wrap, valid, has_normal, normals32, thr=(0.2, 0.2, 0.2), predicate=0, cos_min=0.0):
    """Step 5 (Algorithm 1) on a grid: labels per cell (0 = empty cell), K.
    predicate 0: component-wise thresholds thr; 1: n_p . n_q > cos_min."""
    valid = _c(valid, np.uint8)
    has_normal = _c(has_normal, np.uint8)
    normals32 = _c(normals32, np.float32).reshape(-1, 3)
    thr = _c(thr, np.float64)
    out = np.empty(H * Wp, dtype=np.int32)
    K = lib().oracle_labels_pred(H, Wp, wrap, _p(valid), _p(has_normal), _p(normals32), int(predicate),
                                 _p(thr), float(cos_min), _p(out))
    return out, int(K)


def prune(vertex_labels, K, min_size):
    """Step 6a: labels carried by fewer than min_size vertices become 0."""
    out = _c(vertex_labels, np.int32).copy()
    lib().oracle_prune(_p(out), out.shape[0], int(K), int(min_size))
    return out


def point_cells(xyz, H, W, elev, az0=0.0, r_min=1.0, r_max=60.0, ring_ids=None):
    """Every point's full-resolution (ring, firing), -1 for a point that is not used."""
    xyz = _c(xyz, np.float32).reshape(-1, 3)
    elev = _c(elev, np.float64)
    rk, rp = _rings(ring_ids, xyz.shape[0])
    ring = np.empty(xyz.shape[0], np.int32)
    firing = np.empty(xyz.shape[0], np.int32)
    lib().oracle_point_cells(_p(xyz), rp, xyz.shape[0], H, W, _p(elev), az0, r_min, r_max, _p(ring), _p(firing))
    return ring, firing


def backfill(ring, firing, H, W, s, wrap, cell_label):
    """Step 6b: every point's label from the nearest vertex of its ring along the sweep.
    cell_label: [H * W/s] label of each cell's vertex, -1 for an empty cell."""
    ring = _c(ring, np.int32)
    firing = _c(firing, np.int32)
    cell_label = _c(cell_label, np.int32)
    out = np.empty(ring.shape[0], np.int32)
    lib().oracle_backfill(ring.shape[0], _p(ring), _p(firing), H, W, s, wrap, _p(cell_label), _p(out))
    return out


def edge_scores(H, Wp, wrap, cell_label, cell_truth, radius=1):
    """Step 7: (segment edges, truth edges, found, recalled) of a labelled lattice.
    cell_label: [H * Wp] label of each cell's vertex, -1 for an empty cell;
    cell_truth: [H * Wp] ground-truth surface id of each cell's vertex."""
    cell_label = _c(cell_label, np.int32)
    cell_truth = _c(cell_truth, np.int32)
    out = np.zeros(4, np.int64)
    lib().oracle_edge_scores(H, Wp, wrap, _p(cell_label), _p(cell_truth), int(radius), _p(out))
    return tuple(int(x) for x in out)


def precision_recall_f1(counts):
    """Precision, recall and F1 from edge counts; a side with no edges scores 1
    when the other has none either, else 0."""
    n_seg, n_tru, found, recalled = counts
    p = found / n_seg if n_seg else (1.0 if n_tru == 0 else 0.0)
    r = recalled / n_tru if n_tru else (1.0 if n_seg == 0 else 0.0)
    f = 2 * p * r / (p + r) if p + r > 0 else 0.0
    return p, r, f


def frame_edge_scores(xyz, truth, H, W, s, elev, labels, *, az0=0.0, r_min=1.0, r_max=60.0, wrap=1, radius=1):
    """Edge counts of one sweep's vertex labels (vertex order) against the
    per-point truth ids, through the sweep's own binning."""
    cp = bin_points(xyz, H, W, s, elev, az0, r_min, r_max)
    used = cp >= 0
    cell_label = np.full(cp.shape[0], -1, np.int32)
    cell_truth = np.full(cp.shape[0], -1, np.int32)
    cell_label[used] = np.asarray(labels, np.int32)
    cell_truth[used] = np.asarray(truth, np.int32)[cp[used]]
    return edge_scores(H, W // s, wrap, cell_label, cell_truth, radius)


@dataclass
class Result:
    vertices: np.ndarray      # float32 [V,3]
    normals: np.ndarray       # float32 [V,3]
    labels: np.ndarray        # int32 [V]
    triangles: np.ndarray     # int32 [T,3]
    vertex_point: np.ndarray  # int32 [V]
    normals64: np.ndarray     # float64 [V,3]
    point_labels: np.ndarray | None = None  # int32 [N] (when asked for)
    K: int | None = None      # label count before segment removal

    @property
    def counts(self):
        K = self.K if self.K is not None else (int(self.labels.max()) if self.labels.size else 0)
        return (self.vertices.shape[0], self.triangles.shape[0], K)


def mesh_segment(xyz, H, W, s, elev, *, az0=0.0, r_min=1.0, r_max=60.0, thr=(0.2, 0.2, 0.2),
                 wrap=1, predicate=0, cos_min=0.0, min_segment=0, point_labels=False, ring_ids=None) -> Result:
    """The whole path on one sweep (compact outputs in vertex order); with
    point_labels, every input point's label as well (step 6b); ring_ids: each
    point's reported ring instead of the elevation decision."""
    xyz = _c(xyz, np.float32).reshape(-1, 3)
    rk, rp = _rings(ring_ids, xyz.shape[0])
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
    PL = np.empty(max(xyz.shape[0], 1), np.int32) if point_labels else None
    cnt = np.zeros(3, np.int64)
    rc = lib().oracle_mesh_segment_ex(_p(xyz), rp, xyz.shape[0], H, W, s, wrap, _p(elev), az0, r_min, r_max,
                                      int(predicate), _p(thr), float(cos_min), int(min_segment), _p(V), _p(Nn),
                                      _p(L), _p(T), _p(VP), _p(cnt), _p(N64), _p(PL) if PL is not None else None)
    if rc != 0:
        raise ValueError("oracle_mesh_segment: bad arguments")
    v, t = int(cnt[0]), int(cnt[1])
    return Result(V[:v].copy(), Nn[:v].copy(), L[:v].copy(), T[:t].copy(), VP[:v].copy(), N64[:v].copy(),
                  PL[:xyz.shape[0]].copy() if PL is not None else None, int(cnt[2]))


def mesh_segment_frame(frame, s=1, **kw) -> Result:
    """Convenience: run on a synth.Frame."""
    sen = frame.sensor
    return mesh_segment(frame.xyz, sen.n_rings, sen.n_azimuth, s, sen.elevations(), az0=sen.az0, **kw)
