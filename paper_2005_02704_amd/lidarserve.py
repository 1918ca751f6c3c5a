"""Thin ctypes binding of the native served form (include/lidarserve.h).

The scheduler, the server thread, the copies and the launches all run inside
liblidarseg.so; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .lidarseg import (LAUNCH, LIDAR_OK, LidarError, SensorGeometry, lidar_params_t, lidar_sensor_t,
                       load_library, make_params)

SERVE_EXPORTS = ("lidar_server_create", "lidar_server_destroy", "lidar_server_last_error", "lidar_server_now",
                 "lidar_server_submit", "lidar_server_poll", "lidar_server_result", "lidar_server_release",
                 "lidar_server_stats", "lidar_server_replay")
LIDAR_SERVED_OK = 2
LIDAR_SERVED_TIMED_OUT = 3
LIDAR_SERVED_FAILED = 4


class lidar_server_opts_t(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("sets_per_sensor", ctypes.c_int32), ("budget_bytes", ctypes.c_uint64), ("timeout_s", ctypes.c_double),
                ("copy_mesh", ctypes.c_int32), ("tile_cells", ctypes.c_int32), ("tile_threads", ctypes.c_int32),
                ("grid", ctypes.c_int32)]


class lidar_served_t(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("sensor", ctypes.c_int32), ("status", ctypes.c_int32),
                ("slot", ctypes.c_int32), ("group_size", ctypes.c_int32), ("t_arrival", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class lidar_server_result_t(ctypes.Structure):
    _fields_ = [("counts", ctypes.POINTER(ctypes.c_int64)), ("labels", ctypes.POINTER(ctypes.c_int32)),
                ("vertex_point", ctypes.POINTER(ctypes.c_int32)), ("vertices", ctypes.POINTER(ctypes.c_float)),
                ("normals", ctypes.POINTER(ctypes.c_float)), ("triangles", ctypes.POINTER(ctypes.c_int32))]


class lidar_server_stats_t(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_int64), ("admitted", ctypes.c_int64), ("timed_out", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("peak_bytes", ctypes.c_uint64), ("max_slots_busy", ctypes.c_int32),
                ("device_bytes", ctypes.c_uint64)]


def _bind(L):
    if getattr(L, "_serve_bound", False):
        return L
    P = ctypes.c_void_p
    L.lidar_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(lidar_sensor_t), ctypes.c_int32,
                                      ctypes.POINTER(lidar_params_t), ctypes.POINTER(lidar_server_opts_t),
                                      ctypes.POINTER(P)]
    L.lidar_server_create.restype = ctypes.c_int
    L.lidar_server_destroy.argtypes = [P]
    L.lidar_server_destroy.restype = None
    L.lidar_server_last_error.argtypes = [P]
    L.lidar_server_last_error.restype = ctypes.c_char_p
    L.lidar_server_now.argtypes = [P]
    L.lidar_server_now.restype = ctypes.c_double
    L.lidar_server_submit.argtypes = [P, ctypes.c_int32, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.lidar_server_submit.restype = ctypes.c_int
    L.lidar_server_poll.argtypes = [P, ctypes.POINTER(lidar_served_t), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.lidar_server_poll.restype = ctypes.c_int
    L.lidar_server_result.argtypes = [P, ctypes.c_int64, ctypes.POINTER(lidar_server_result_t)]
    L.lidar_server_result.restype = ctypes.c_int
    L.lidar_server_release.argtypes = [P, ctypes.c_int64]
    L.lidar_server_release.restype = ctypes.c_int
    L.lidar_server_stats.argtypes = [P, ctypes.POINTER(lidar_server_stats_t)]
    L.lidar_server_stats.restype = ctypes.c_int
    L.lidar_server_replay.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P, P, ctypes.POINTER(ctypes.c_double)]
    L.lidar_server_replay.restype = ctypes.c_int
    L._serve_bound = True
    return L


class NativeServer:
    """A lidar_server: the continuous-batching server of liblidarseg.

    sensors: [SensorGeometry]; requests name a sensor by index.  Host points
    given to submit() should be pinned; the binding holds them until poll()
    reports the request finished (until close() for a request that timed out,
    whose group may still read them)."""

    def __init__(self, sensors, device: int = 0, params=None, n_slots: int = 3, max_batch: int = 64,
                 launch: str = "graph", sets_per_sensor: int = 16, budget_bytes: int = 1 << 30,
                 timeout_s: float = 0.0, copy_mesh: bool = False, tile_cells: int = 0, tile_threads: int = 0,
                 grid: int = 0):
        self._L = _bind(load_library())
        self.sensors = list(sensors)
        n = len(self.sensors)
        arr = (lidar_sensor_t * n)()
        for q, g in enumerate(self.sensors):
            arr[q] = g.c_struct()   # the server copies the geometry, elevations included
        self._params = params or make_params()
        opts = lidar_server_opts_t(n_slots, max_batch, LAUNCH[launch] if isinstance(launch, str) else int(launch),
                                   sets_per_sensor, int(budget_bytes), float(timeout_s), 1 if copy_mesh else 0,
                                   tile_cells, tile_threads, grid)
        self._h = ctypes.c_void_p()
        rc = self._L.lidar_server_create(device, arr, n, ctypes.byref(self._params), ctypes.byref(opts),
                                         ctypes.byref(self._h))
        if rc != LIDAR_OK:
            raise LidarError(rc, self._L.lidar_server_last_error(None).decode())
        self.copy_mesh = copy_mesh
        self._held = {}       # request id -> host points kept alive until it finishes
        self._abandoned = []  # points of timed-out requests: their group may still read them

    def close(self):
        if self._h:
            self._L.lidar_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._held.clear()
            self._abandoned.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != LIDAR_OK:
            raise LidarError(rc, self._L.lidar_server_last_error(self._h).decode())

    def now(self) -> float:
        return self._L.lidar_server_now(self._h)

    def submit(self, sensor: int, xyz, n_points: int | None = None) -> int:
        """xyz: host float32 [N, 3] (numpy array or pinned torch tensor)."""
        ptr = xyz.data_ptr() if hasattr(xyz, "data_ptr") else xyz.ctypes.data
        n = int(xyz.shape[0]) if n_points is None else int(n_points)
        rid = ctypes.c_int64()
        self._check(self._L.lidar_server_submit(self._h, int(sensor), ctypes.c_void_p(ptr if n else None), n,
                                                ctypes.byref(rid)))
        self._held[rid.value] = xyz
        return rid.value

    def poll(self, max_n: int = 256):
        """Finished requests: [dict(id, sensor, status, slot, group_size, t_arrival, t_admit, t_done)]."""
        buf = (lidar_served_t * max_n)()
        k = ctypes.c_int32()
        self._check(self._L.lidar_server_poll(self._h, buf, max_n, ctypes.byref(k)))
        out = []
        for d in buf[:k.value]:
            pts = self._held.pop(d.id, None)
            if d.status == LIDAR_SERVED_TIMED_OUT:
                self._abandoned.append(pts)
            out.append(dict(id=d.id, sensor=d.sensor, status=d.status, slot=d.slot, group_size=d.group_size,
                            t_arrival=d.t_arrival, t_admit=d.t_admit, t_done=d.t_done))
        return out

    def result(self, rid: int):
        """Copies of a served request's results (counts, labels, vertex_point,
        and with copy_mesh vertices, normals, triangles)."""
        r = lidar_server_result_t()
        self._check(self._L.lidar_server_result(self._h, int(rid), ctypes.byref(r)))
        V, T, K = (int(r.counts[j]) for j in range(3))
        out = dict(counts=(V, T, K),
                   labels=np.ctypeslib.as_array(r.labels, shape=(max(V, 1),))[:V].copy(),
                   vertex_point=np.ctypeslib.as_array(r.vertex_point, shape=(max(V, 1),))[:V].copy())
        if self.copy_mesh:
            out["vertices"] = np.ctypeslib.as_array(r.vertices, shape=(max(V, 1), 3))[:V].copy()
            out["normals"] = np.ctypeslib.as_array(r.normals, shape=(max(V, 1), 3))[:V].copy()
            out["triangles"] = np.ctypeslib.as_array(r.triangles, shape=(max(T, 1), 3))[:T].copy()
        return out

    def release(self, rid: int):
        self._check(self._L.lidar_server_release(self._h, int(rid)))

    def stats(self):
        st = lidar_server_stats_t()
        self._check(self._L.lidar_server_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def replay(self, t_offset, sensor, xyz_list, n_points=None):
        """Native benchmark driver: request i submitted t_offset[i] s after the
        start; returns (latency_s, status, group_size, wall_s)."""
        n = len(t_offset)
        t = np.ascontiguousarray(t_offset, np.float64)
        s = np.ascontiguousarray(sensor, np.int32)
        ptrs = np.array([x.data_ptr() if hasattr(x, "data_ptr") else x.ctypes.data for x in xyz_list], np.uint64)
        npts = np.ascontiguousarray([int(x.shape[0]) for x in xyz_list] if n_points is None else n_points, np.int64)
        lat = np.zeros(n, np.float64)
        st = np.zeros(n, np.int32)
        gs = np.zeros(n, np.int32)
        wall = ctypes.c_double()
        self._check(self._L.lidar_server_replay(self._h, n, t.ctypes.data, s.ctypes.data, ptrs.ctypes.data,
                                                npts.ctypes.data, lat.ctypes.data, st.ctypes.data, gs.ctypes.data,
                                                ctypes.byref(wall)))
        return lat, st, gs, wall.value
