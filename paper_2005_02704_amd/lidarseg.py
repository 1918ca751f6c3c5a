"""Thin ctypes binding of liblidarseg (include/lidarseg.h).

Argument marshalling only: every stage of the path runs in the HIP library.
PyTorch supplies device memory (tensors) and streams.  The binding refuses to
run without the built library; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblidarseg.so")

LIDAR_OK = 0
LIDAR_EINVAL = -1
LIDAR_ENOMEM = -2
LIDAR_EDEVICE = -3
LIDAR_MAX_RINGS = 128

LIDAR_LAUNCH_PLAIN = 0
LIDAR_LAUNCH_BATCHED = 1
LIDAR_LAUNCH_GRAPH = 2
LAUNCH = {"plain": LIDAR_LAUNCH_PLAIN, "batched": LIDAR_LAUNCH_BATCHED, "graph": LIDAR_LAUNCH_GRAPH}
LIDAR_PRED_COMPONENTS = 0
LIDAR_PRED_COSINE = 1

# every symbol include/lidarseg.h declares
EXPORTS = ("lidar_ctx_create", "lidar_ctx_destroy", "lidar_ctx_last_error", "lidar_last_error",
           "lidar_query_sizes", "lidar_mesh_segment", "lidar_mesh_normals", "lidar_label_grid",
           "lidar_ctx_set_workspace_limit", "lidar_ctx_workspace_bytes", "lidar_ctx_set_tuning",
           "lidar_ctx_set_stage_grid",
           "lidar_ctx_set_profiling", "lidar_ctx_stage_times", "lidar_mesh_segment_noalloc")
LIDAR_N_STAGES = 11
STAGES = ("bin", "count", "geom", "cc", "merge", "compress", "flatten", "scan", "label", "post", "score")
LIDAR_MAX_SCORE_RADIUS = 8
LIDAR_NOALLOC_SCRATCH_BYTES = 64 << 20
LIDAR_NOALLOC_MAX_FRAMES = 64


class LidarError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblidarseg error {code}: {msg}")
        self.code = code


class lidar_sensor_t(ctypes.Structure):
    _fields_ = [("n_rings", ctypes.c_int32), ("n_azimuth", ctypes.c_int32),
                ("subsample", ctypes.c_int32), ("wrap", ctypes.c_int32),
                ("elev_rad", ctypes.POINTER(ctypes.c_double)), ("az0_rad", ctypes.c_double)]


class lidar_frame_t(ctypes.Structure):
    _fields_ = [("sensor", ctypes.POINTER(lidar_sensor_t)), ("xyz", ctypes.c_void_p),
                ("n_points", ctypes.c_int64), ("normals_in", ctypes.c_void_p), ("truth_ids", ctypes.c_void_p),
                ("ring_ids", ctypes.c_void_p)]


class lidar_params_t(ctypes.Structure):
    _fields_ = [("r_min", ctypes.c_double), ("r_max", ctypes.c_double), ("thr", ctypes.c_double * 3),
                ("predicate", ctypes.c_int32), ("min_segment", ctypes.c_int32), ("cos_min", ctypes.c_double),
                ("score_radius", ctypes.c_int32)]


class lidar_result_t(ctypes.Structure):
    _fields_ = [("vertices", ctypes.c_void_p), ("normals", ctypes.c_void_p),
                ("labels", ctypes.c_void_p), ("triangles", ctypes.c_void_p),
                ("vertex_point", ctypes.c_void_p), ("counts", ctypes.c_void_p),
                ("point_labels", ctypes.c_void_p), ("edge_counts", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblidarseg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2005_02704_amd/build.py "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    L.lidar_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
    L.lidar_ctx_create.restype = ctypes.c_int
    L.lidar_ctx_destroy.argtypes = [P]
    L.lidar_ctx_destroy.restype = None
    L.lidar_ctx_last_error.argtypes = [P]
    L.lidar_ctx_last_error.restype = ctypes.c_char_p
    L.lidar_last_error.argtypes = []
    L.lidar_last_error.restype = ctypes.c_char_p
    L.lidar_query_sizes.argtypes = [ctypes.POINTER(lidar_sensor_t), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64)]
    L.lidar_query_sizes.restype = ctypes.c_int
    L.lidar_mesh_segment.argtypes = [P, ctypes.POINTER(lidar_frame_t), ctypes.c_int32,
                                     ctypes.POINTER(lidar_params_t), ctypes.POINTER(lidar_result_t),
                                     P, ctypes.c_int32]
    L.lidar_mesh_segment.restype = ctypes.c_int
    for name in ("lidar_mesh_normals", "lidar_label_grid", "lidar_mesh_segment_noalloc"):
        getattr(L, name).argtypes = L.lidar_mesh_segment.argtypes
        getattr(L, name).restype = ctypes.c_int
    L.lidar_ctx_set_workspace_limit.argtypes = [P, ctypes.c_uint64]
    L.lidar_ctx_set_workspace_limit.restype = ctypes.c_int
    L.lidar_ctx_workspace_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_uint64)]
    L.lidar_ctx_workspace_bytes.restype = ctypes.c_int
    L.lidar_ctx_set_stage_grid.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    L.lidar_ctx_set_stage_grid.restype = ctypes.c_int
    L.lidar_ctx_set_tuning.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.lidar_ctx_set_tuning.restype = ctypes.c_int
    L.lidar_ctx_set_profiling.argtypes = [P, ctypes.c_int32]
    L.lidar_ctx_set_profiling.restype = ctypes.c_int
    L.lidar_ctx_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.lidar_ctx_stage_times.restype = ctypes.c_int
    _lib = L
    return L


@dataclass
class SensorGeometry:
    """Host description of a sensor: ring elevations (radians, descending), firings, s."""
    elev_rad: np.ndarray
    n_azimuth: int
    subsample: int = 1
    wrap: int = 1
    az0_rad: float = 0.0
    _c: lidar_sensor_t = field(default=None, repr=False)
    _elev: np.ndarray = field(default=None, repr=False)

    @property
    def n_rings(self) -> int:
        return int(len(self.elev_rad))

    @property
    def n_cols(self) -> int:
        return self.n_azimuth // self.subsample

    def c_struct(self) -> lidar_sensor_t:
        if self._c is None:
            self._elev = np.ascontiguousarray(self.elev_rad, dtype=np.float64)
            self._c = lidar_sensor_t(self.n_rings, int(self.n_azimuth), int(self.subsample), int(self.wrap),
                                     self._elev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     float(self.az0_rad))
        return self._c


def lidar_query_sizes(sensor: SensorGeometry):
    L = load_library()
    v = ctypes.c_int64()
    t = ctypes.c_int64()
    rc = L.lidar_query_sizes(ctypes.byref(sensor.c_struct()), ctypes.byref(v), ctypes.byref(t))
    if rc != LIDAR_OK:
        raise LidarError(rc, L.lidar_last_error().decode())
    return int(v.value), int(t.value)


class Outputs:
    """Caller-owned device outputs of one frame (torch tensors at full capacity)."""

    def __init__(self, sensor: SensorGeometry, device, with_vertex_point=True, n_points: int = 0,
                 scores: bool = False, with_labels: bool = True):
        """n_points > 0 also allocates point_labels (every input point's label);
        scores allocates edge_counts (edge scores against the frame's truth ids);
        with_labels=False leaves labels out (lidar_mesh_normals writes none)."""
        import torch
        V, T = lidar_query_sizes(sensor)
        self.vertices = torch.empty((max(V, 1), 3), dtype=torch.float32, device=device)
        self.normals = torch.empty((max(V, 1), 3), dtype=torch.float32, device=device)
        self.labels = torch.empty(max(V, 1), dtype=torch.int32, device=device) if with_labels else None
        self.triangles = torch.empty((max(T, 1), 3), dtype=torch.int32, device=device)
        self.vertex_point = torch.empty(max(V, 1), dtype=torch.int32, device=device) if with_vertex_point else None
        self.counts = torch.zeros(3, dtype=torch.int64, device=device)
        self.point_labels = torch.empty(n_points, dtype=torch.int32, device=device) if n_points > 0 else None
        self.edge_counts = torch.zeros(4, dtype=torch.int64, device=device) if scores else None

    def c_struct(self) -> lidar_result_t:
        return lidar_result_t(self.vertices.data_ptr(), self.normals.data_ptr(),
                              self.labels.data_ptr() if self.labels is not None else None,
                              self.triangles.data_ptr(),
                              self.vertex_point.data_ptr() if self.vertex_point is not None else None,
                              self.counts.data_ptr(),
                              self.point_labels.data_ptr() if self.point_labels is not None else None,
                              self.edge_counts.data_ptr() if self.edge_counts is not None else None)

    def trimmed(self):
        """Views cut to the counts (synchronises with the device to read them)."""
        V, T, K = (int(x) for x in self.counts.cpu())
        if V < 0 or T < 0 or K < 0:
            raise LidarError(LIDAR_EDEVICE, "the frame's device work failed (counts = -1)")
        return dict(vertices=self.vertices[:V], normals=self.normals[:V],
                    labels=self.labels[:V] if self.labels is not None else None,
                    triangles=self.triangles[:T],
                    vertex_point=self.vertex_point[:V] if self.vertex_point is not None else None,
                    point_labels=self.point_labels, counts=(V, T, K),
                    edge_counts=tuple(int(x) for x in self.edge_counts.cpu()) if self.edge_counts is not None
                    else None)


def check_tensor(name, t, device, dtype, min_rows, cols=None, optional=False):
    """Refuse (LidarError, LIDAR_EINVAL) a tensor the library could not read or
    write safely: not on `device`, not contiguous, of another dtype, with fewer
    than min_rows rows, or (cols given) not [rows, cols].  Nothing is launched."""
    if t is None:
        if optional:
            return
        raise LidarError(LIDAR_EINVAL, f"{name} is required")
    if t.device != device:
        raise LidarError(LIDAR_EINVAL, f"{name} is on {t.device}, not {device}")
    if t.dtype != dtype:
        raise LidarError(LIDAR_EINVAL, f"{name} is {t.dtype}, not {dtype}")
    if not t.is_contiguous():
        raise LidarError(LIDAR_EINVAL, f"{name} is not contiguous")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise LidarError(LIDAR_EINVAL, f"{name} has shape {tuple(t.shape)}, not [rows, {cols}]")
    if cols is None and t.dim() != 1:
        raise LidarError(LIDAR_EINVAL, f"{name} has shape {tuple(t.shape)}, not [rows]")
    rows = t.shape[0]
    if rows < min_rows:
        raise LidarError(LIDAR_EINVAL, f"{name} has {rows} rows, needs at least {min_rows}")


def check_frame(device, xyz, sensor, normals_in, truth, rings, out, n_points=None):
    """Every tensor of one frame against what the library reads and writes:
    xyz float32 [N, 3]; normals_in float32 [>= max_vertices, 3]; truth ids int32
    [N]; reported rings uint8 [N]; outputs at the capacities lidar_query_sizes
    gives (vertices and normals float32 [V, 3], labels and vertex_point int32 [V],
    triangles int32 [T, 3], counts int64 [3], point_labels int32 [N], edge counts
    int64 [4]).  V, T = max_vertices, max_triangles of the sensor."""
    import torch
    check_tensor("xyz", xyz, device, torch.float32, 0, 3)
    N = int(xyz.shape[0])
    V, T = lidar_query_sizes(sensor)
    check_tensor("normals_in", normals_in, device, torch.float32, V, 3, optional=True)
    check_tensor("truth_ids", truth, device, torch.int32, N, optional=True)
    check_tensor("ring_ids", rings, device, torch.uint8, N, optional=True)
    check_tensor("vertices", out.vertices, device, torch.float32, V, 3)
    check_tensor("normals", out.normals, device, torch.float32, V, 3)
    check_tensor("labels", out.labels, device, torch.int32, V, optional=True)
    check_tensor("triangles", out.triangles, device, torch.int32, T, 3)
    check_tensor("vertex_point", out.vertex_point, device, torch.int32, V, optional=True)
    check_tensor("counts", out.counts, device, torch.int64, 3)
    check_tensor("point_labels", out.point_labels, device, torch.int32, N, optional=True)
    check_tensor("edge_counts", out.edge_counts, device, torch.int64, 4, optional=True)


class LidarContext:
    """A lidar_ctx: device workspace and captured graph, used by one thread at a time."""

    def __init__(self, device: int = 0):
        self._L = load_library()
        self._h = ctypes.c_void_p()
        rc = self._L.lidar_ctx_create(int(device), ctypes.byref(self._h))
        if rc != LIDAR_OK:
            raise LidarError(rc, self._L.lidar_last_error().decode())
        self.device = device

    def close(self):
        if self._h:
            self._L.lidar_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, grid_workgroups: int = 0, tile_cells: int = 0, tile_threads: int = 0):
        rc = self._L.lidar_ctx_set_tuning(self._h, int(grid_workgroups), int(tile_cells), int(tile_threads))
        self._check(rc)

    def set_stage_grid(self, stage, workgroups: int = 0):
        """Workgroups of one stage (name from STAGES, or index) in batched and graph
        launches; 0 = its share of the tuning grid."""
        k = STAGES.index(stage) if isinstance(stage, str) else int(stage)
        self._check(self._L.lidar_ctx_set_stage_grid(self._h, k, int(workgroups)))

    def set_profiling(self, enable: bool):
        self._check(self._L.lidar_ctx_set_profiling(self._h, 1 if enable else 0))

    def stage_times(self):
        """{stage: (total_ms, launches)} since the last call; waits for the timed work."""
        ms = (ctypes.c_double * LIDAR_N_STAGES)()
        n = (ctypes.c_int64 * LIDAR_N_STAGES)()
        self._check(self._L.lidar_ctx_stage_times(self._h, ms, n))
        return {name: (float(ms[k]), int(n[k])) for k, name in enumerate(STAGES)}

    def _check(self, rc):
        if rc != LIDAR_OK:
            raise LidarError(rc, self._L.lidar_ctx_last_error(self._h).decode())

    def prepare(self, inputs, params: lidar_params_t, outputs):
        """Build the C argument arrays once (for repeated launches on the same buffers)."""
        import torch
        n = len(inputs)
        if len(outputs) != n:
            raise LidarError(LIDAR_EINVAL, f"{n} inputs but {len(outputs)} outputs")
        dev = torch.device("cuda", self.device)
        frames = (lidar_frame_t * n)()
        results = (lidar_result_t * n)()
        keep = []
        for f, item in enumerate(inputs):
            xyz, sensor, normals_in = item[:3]
            truth = item[3] if len(item) > 3 else None
            rings = item[4] if len(item) > 4 else None
            try:
                check_frame(dev, xyz, sensor, normals_in, truth, rings, outputs[f])
            except LidarError as err:
                raise LidarError(err.code, f"frame {f}: {err}") from None
            sc = sensor.c_struct()
            # the struct points into the geometry's own elevation array, so the
            # prepared call holds the geometry as well as the struct
            keep.append((sensor, sc))
            frames[f] = lidar_frame_t(ctypes.pointer(sc), xyz.data_ptr() if xyz.numel() else None,
                                      int(xyz.shape[0]),
                                      normals_in.data_ptr() if normals_in is not None else None,
                                      truth.data_ptr() if truth is not None and truth.numel() else None,
                                      rings.data_ptr() if rings is not None and rings.numel() else None)
            results[f] = outputs[f].c_struct()
            # the prepared call holds the tensors whose pointers it carries, so
            # none of them is freed (and its memory reused) while the call lives
            keep.append((xyz, normals_in, truth, rings, outputs[f]))
        return (frames, n, params, results, keep, set())

    def _call(self, fn, prepared, stream, launch):
        import torch
        frames, n, params, results, keep, recorded = prepared
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        mode = LAUNCH[launch] if isinstance(launch, str) else int(launch)
        if stream.cuda_stream not in recorded:
            # torch's caching allocator reuses a freed tensor's memory once the
            # stream it was allocated on has passed the free; a call on another
            # stream is made known to it, so no buffer of the call is handed out
            # again while the call may still read or write it (once per stream:
            # the allocator waits on every recorded stream when the tensor is freed)
            for item in keep:
                if isinstance(item, tuple) and len(item) == 5:
                    xyz, normals_in, truth, rings, out = item
                    for t in (xyz, normals_in, truth, rings, out.vertices, out.normals, out.labels,
                              out.triangles, out.vertex_point, out.counts, out.point_labels, out.edge_counts):
                        if t is not None and t.numel():
                            t.record_stream(stream)
            recorded.add(stream.cuda_stream)
        self._check(fn(self._h, frames, n, ctypes.byref(params), results, ctypes.c_void_p(stream.cuda_stream), mode))

    def lidar_mesh_segment(self, prepared, stream=None, launch: str | int = "batched"):
        """Enqueue lidar_mesh_segment on `stream` (torch stream; default: current)."""
        self._call(self._L.lidar_mesh_segment, prepared, stream, launch)

    def lidar_mesh_normals(self, prepared, stream=None, launch: str | int = "batched"):
        """Enqueue lidar_mesh_normals (binning, mesh and normals; no labels)."""
        self._call(self._L.lidar_mesh_normals, prepared, stream, launch)

    def lidar_label_grid(self, prepared, stream=None, launch: str | int = "batched"):
        """Enqueue lidar_label_grid (labels of caller-given normals)."""
        self._call(self._L.lidar_label_grid, prepared, stream, launch)

    def lidar_mesh_segment_noalloc(self, prepared, stream=None, launch: str | int = "batched"):
        """Enqueue lidar_mesh_segment_noalloc (plain or batched; workspace in the
        GPU's fixed scratch array, nothing allocated by the library)."""
        self._call(self._L.lidar_mesh_segment_noalloc, prepared, stream, launch)

    def set_workspace_limit(self, max_bytes: int):
        """Device workspace bytes this context may hold (0 = no limit)."""
        self._check(self._L.lidar_ctx_set_workspace_limit(self._h, int(max_bytes)))

    def workspace_bytes(self) -> int:
        """Device workspace bytes the context holds now."""
        v = ctypes.c_uint64()
        self._check(self._L.lidar_ctx_workspace_bytes(self._h, ctypes.byref(v)))
        return int(v.value)


def make_params(r_min=1.0, r_max=60.0, thr=(0.2, 0.2, 0.2), predicate=LIDAR_PRED_COMPONENTS, cos_min=0.0,
                min_segment=0, score_radius=1) -> lidar_params_t:
    return lidar_params_t(float(r_min), float(r_max), (ctypes.c_double * 3)(*[float(t) for t in thr]),
                          int(predicate), int(min_segment), float(cos_min), int(score_radius))


def precision_recall_f1(edge_counts):
    """Precision, recall and F1 of one frame's edge counts (segment edges, truth
    edges, found, recalled); a side without edges scores 1 when the other has
    none either, else 0."""
    n_seg, n_tru, found, recalled = (int(x) for x in edge_counts)
    p = found / n_seg if n_seg else (1.0 if n_tru == 0 else 0.0)
    r = recalled / n_tru if n_tru else (1.0 if n_seg == 0 else 0.0)
    return p, r, (2 * p * r / (p + r) if p + r > 0 else 0.0)


def lidar_mesh_segment(ctx: LidarContext, inputs, params: lidar_params_t | None = None,
                       launch: str = "batched", stream=None, with_vertex_point=True, point_labels=False,
                       scores=False):
    """Convenience: inputs = [(xyz cuda float32 [N,3], SensorGeometry, normals_in or None
    [, truth ids cuda int32 [N] or None [, reported rings cuda uint8 [N]]])]; scores asks
    for the edge counts (needs truth ids).

    Allocates outputs, enqueues the call and returns the Outputs objects (call
    .trimmed() to synchronise and cut them to their counts)."""
    import torch
    params = params or make_params()
    dev = torch.device("cuda", ctx.device)
    outs = [Outputs(item[1], dev, with_vertex_point, int(item[0].shape[0]) if point_labels else 0, scores)
            for item in inputs]
    if stream is not None:
        # the outputs were made (counts zero-filled) on the current stream
        stream.wait_stream(torch.cuda.current_stream(dev))
    prep = ctx.prepare(inputs, params, outs)
    ctx.lidar_mesh_segment(prep, stream=stream, launch=launch)
    return outs
