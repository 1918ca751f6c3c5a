"""Continuous-batching server for sweeps from several sensors.

Requests (one sweep each) arrive over time.  A scheduler loop admits waiting
requests into free *slots* -- each slot is one lidar context with its own HIP
stream -- as long as the device-memory budget allows, launches each admitted
group as one batched call, and completes requests as their slot's work finishes.
Requests that arrive while other groups are on the GPU join the next free slot,
so several groups overlap on the device.  Per-sensor device buffers (points in,
mesh and labels out) and pinned host buffers stay resident and are reused.

The executor is pluggable: `GpuExecutor` drives liblidarseg; tests drive the
same scheduler with a fake executor on the CPU.
"""
from __future__ import annotations

import collections
import heapq
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    sensor: int            # sensor index (selects geometry and resident buffers)
    xyz: object            # host points: numpy float32 [N,3] or pinned torch tensor
    n_points: int
    t_arrival: float       # host clock (time.perf_counter) when the sweep arrived
    t_admit: float = 0.0
    t_done: float = 0.0
    slot: int = -1
    batch_id: int = -1
    batch_size: int = 0
    result: dict | None = None
    failed: str = ""       # why the request failed (empty: served)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class SlotState:
    busy: bool = False
    handle: object = None
    batch: list = field(default_factory=list)
    bytes_held: int = 0
    t_submit: float = 0.0
    abandoned: bool = False  # its tickets failed on the watchdog; the device work still runs


class Server:
    """Scheduler: admission by slot and memory budget, FIFO, continuous batching.

    executor must provide:
      n_slots                       number of independent launch slots
      bytes_for(req) -> int         device bytes a request needs while in flight
      submit(slot, reqs) -> handle  enqueue the group; returns at once
      poll(handle) -> bool          True once the group's outputs are on the host
      results(handle) -> list       per-request result dicts (after poll is True);
                                    the group's buffers go back to their pools
      discard(handle)               (after poll is True) the group's buffers go back
                                    to their pools without reading its results

    timeout_s: a watchdog on each group.  A group still running that long after
    submission fails its requests (failed = "timeout"; they are finished and
    counted, without results), so callers are never left waiting.  Its slot and
    memory stay held until the device work really completes (the work may
    still write into them), and are then released silently: the executor
    discards the group, returning its buffers to their pools.
    """

    def __init__(self, executor, budget_bytes: int, max_batch: int = 64, timeout_s: float | None = None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.timeout_s = timeout_s
        self.failed = 0
        self.slots = [SlotState() for _ in range(executor.n_slots)]
        self.waiting: collections.deque = collections.deque()
        self.in_use = 0
        self.peak_in_use = 0
        self.done: list[Request] = []
        self.batches = 0
        self.max_overlap = 0
        self._lock = threading.Lock()

    # -- admission ----------------------------------------------------------
    def submit(self, req: Request):
        if self.ex.bytes_for(req) > self.budget:
            raise ValueError(f"request {req.rid} needs more device memory than the whole budget")
        with self._lock:
            self.waiting.append(req)

    def _admit(self, now: float):
        for s, st in enumerate(self.slots):
            if st.busy:
                continue
            group, held = [], 0
            with self._lock:
                while self.waiting and len(group) < self.max_batch:
                    need = self.ex.bytes_for(self.waiting[0])
                    if self.in_use + held + need > self.budget:
                        break
                    r = self.waiting.popleft()
                    group.append(r)
                    held += need
            if not group:
                return
            for r in group:
                r.t_admit = now
                r.slot = s
                r.batch_id = self.batches
                r.batch_size = len(group)
            self.batches += 1
            st.busy, st.batch, st.bytes_held = True, group, held
            st.t_submit, st.abandoned = now, False
            self.in_use += held
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            st.handle = self.ex.submit(s, group)
            self.max_overlap = max(self.max_overlap, sum(x.busy for x in self.slots))

    def _complete(self):
        for st in self.slots:
            if not st.busy:
                continue
            if self.ex.poll(st.handle):
                now = time.perf_counter()
                if not st.abandoned:
                    for r, res in zip(st.batch, self.ex.results(st.handle)):
                        r.t_done = now
                        r.result = res
                        self.done.append(r)
                else:
                    self.ex.discard(st.handle)
                self.in_use -= st.bytes_held
                st.busy, st.batch, st.handle, st.bytes_held, st.abandoned = False, [], None, 0, False
            elif (self.timeout_s is not None and not st.abandoned
                  and time.perf_counter() - st.t_submit > self.timeout_s):
                now = time.perf_counter()
                for r in st.batch:
                    r.t_done = now
                    r.failed = "timeout"
                    self.done.append(r)
                self.failed += len(st.batch)
                st.abandoned = True

    def step(self):
        self._complete()
        self._admit(time.perf_counter())

    def idle(self) -> bool:
        """Nothing waiting and no request in flight (an abandoned slot's device
        work may still be running; its requests are already finished)."""
        return not self.waiting and not any(st.busy and not st.abandoned for st in self.slots)

    # -- driving a timed arrival schedule -----------------------------------
    def run_schedule(self, schedule, make_request, poll_sleep: float = 5e-5):
        """schedule: sorted list of (offset_seconds, sensor, payload).  Requests are
        created when their time comes (host arrival = that moment) and served."""
        t0 = time.perf_counter()
        heap = list(schedule)
        heapq.heapify(heap)
        rid = 0
        while heap or not self.idle():
            now = time.perf_counter()
            while heap and heap[0][0] <= now - t0:
                _, sensor, payload = heapq.heappop(heap)
                self.submit(make_request(rid, sensor, payload, time.perf_counter()))
                rid += 1
            self.step()
            if heap and self.idle():
                wait = heap[0][0] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
            elif not self.idle():
                time.sleep(poll_sleep)
        return time.perf_counter() - t0

    # -- statistics ----------------------------------------------------------
    def stats(self, wall_s: float):
        served = [r for r in self.done if not r.failed]
        lat = np.array([r.latency for r in served]) * 1e3
        pts = sum(r.n_points for r in served)
        return {
            "requests": len(served),
            "failed": self.failed,
            "points": int(pts),
            "points_per_s": pts / wall_s if wall_s > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "max_ms": float(lat.max()) if lat.size else None,
            "batches": self.batches,
            "mean_batch": len(self.done) / max(1, self.batches),
            "max_slots_in_flight": self.max_overlap,
            "peak_device_bytes": self.peak_in_use,
        }


def poisson_schedule(rates_hz, seconds: float, seed: int, n_payloads: int):
    """Arrival offsets per sensor: exponential inter-arrival times (Poisson process)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s, rate in enumerate(rates_hz):
        t = rng.exponential(1.0 / rate)
        k = 0
        while t < seconds:
            out.append((float(t), s, k % n_payloads))
            t += rng.exponential(1.0 / rate)
            k += 1
    out.sort()
    return out


class GpuExecutor:
    """Slots = lidar contexts with their own streams; resident per-sensor buffers.

    Each sensor owns a pool of buffer sets (device points, device outputs,
    pinned host copies of labels / vertex_point / counts): sets_per_sensor are
    made up front, more when that many of the sensor's sweeps are in flight at
    once; a set returns to its pool when its results are read and is kept until
    close.  A group is one batched call on its slot's stream: H2D of the points,
    the chain, D2H of the segmentation, then an event the scheduler polls."""

    def __init__(self, geometries, n_slots: int = 3, device: int = 0, launch: str = "batched",
                 params=None, sets_per_sensor: int = 4, copy_mesh: bool = False):
        import torch

        import paper_2005_02704_amd as lp
        self.torch = torch
        self.lp = lp
        self.geos = geometries
        self.n_slots = n_slots
        self.launch = launch
        self.copy_mesh = copy_mesh
        self.dev = torch.device("cuda", device)
        self.params = params or lp.make_params()
        self.ctxs = [lp.LidarContext(device) for _ in range(n_slots)]
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(n_slots)]
        self.sets = [[] for _ in geometries]          # resident buffer sets per sensor
        self.free_sets = [[] for _ in geometries]
        self.caps = [lp.lidar_query_sizes(g) for g in geometries]
        for q in range(len(geometries)):
            for _ in range(sets_per_sensor):
                self.free_sets[q].append(self._new_set(q))
        # the sets made up front are filled on the current stream: finished
        # before any slot stream uses them
        torch.cuda.current_stream(self.dev).synchronize()

    def bytes_for(self, req) -> int:
        V, T = self.caps[req.sensor]
        g = self.geos[req.sensor]
        if req.n_points > g.n_rings * g.n_azimuth:
            # the resident point buffer holds one return per ray
            raise ValueError(f"request {req.rid}: {req.n_points} points, more than the sensor's "
                             f"{g.n_rings * g.n_azimuth} rays")
        cells = g.n_rings * g.n_cols
        return 12 * g.n_rings * g.n_azimuth + 36 * V + 12 * T + 8 * cells + 16 * V

    def _buffer_set(self, sensor):
        if self.free_sets[sensor]:
            return self.free_sets[sensor].pop()
        return self._new_set(sensor)

    def _new_set(self, sensor):
        torch = self.torch
        g = self.geos[sensor]
        V, T = self.caps[sensor]
        Vc = max(V, 1)
        # counts (3 x int64), labels and vertex_point share one device block and
        # one pinned block, so that a sweep's segmentation comes back in one copy:
        # int32 words [0, 6) counts, [8, 8 + Vc) labels, [8 + Vc, 8 + 2 Vc) vertex_point
        d_block = torch.zeros(8 + 2 * Vc, dtype=torch.int32, device=self.dev)
        h_block = torch.empty(8 + 2 * Vc, dtype=torch.int32, pin_memory=True)
        out = self.lp.Outputs(g, self.dev, with_vertex_point=False, with_labels=False)
        out.counts = d_block[0:6].view(torch.int64)
        out.labels = d_block[8:8 + Vc]
        out.vertex_point = d_block[8 + Vc:8 + 2 * Vc]
        bs = dict(
            xyz=torch.empty((g.n_rings * g.n_azimuth, 3), dtype=torch.float32, device=self.dev),
            out=out, d_block=d_block, h_block=h_block, h_np=h_block.numpy(), Vc=Vc,
        )
        if self.copy_mesh:
            bs["h_normals"] = torch.empty((max(V, 1), 3), dtype=torch.float32, pin_memory=True)
            bs["h_vertices"] = torch.empty((max(V, 1), 3), dtype=torch.float32, pin_memory=True)
            bs["h_triangles"] = torch.empty((max(T, 1), 3), dtype=torch.int32, pin_memory=True)
        self.sets[sensor].append(bs)
        return bs

    def submit(self, slot, reqs):
        torch = self.torch
        stream = self.streams[slot]
        inputs, outs = [], []
        with torch.cuda.stream(stream):
            # a set made here (its sensor's pool ran dry) is zero-filled on this
            # slot's stream, so the fill is ordered before the group's kernels
            sets = [self._buffer_set(r.sensor) for r in reqs]
            for r, bs in zip(reqs, sets):
                dst = bs["xyz"][:r.n_points]
                if r.n_points:
                    dst.copy_(r.xyz, non_blocking=True)
                inputs.append((dst, self.geos[r.sensor], None))
                outs.append(bs["out"])
        prep = self.ctxs[slot].prepare(inputs, self.params, outs)
        self.ctxs[slot].lidar_mesh_segment(prep, stream=stream, launch=self.launch)
        with torch.cuda.stream(stream):
            for bs in sets:
                o = bs["out"]
                bs["h_block"].copy_(bs["d_block"], non_blocking=True)
                if self.copy_mesh:
                    bs["h_normals"].copy_(o.normals, non_blocking=True)
                    bs["h_vertices"].copy_(o.vertices, non_blocking=True)
                    bs["h_triangles"].copy_(o.triangles, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return dict(event=ev, reqs=reqs, sets=sets, prep=prep)

    def poll(self, h) -> bool:
        return h["event"].query()

    def results(self, h):
        out = []
        for r, bs in zip(h["reqs"], h["sets"]):
            h, Vc = bs["h_np"], bs["Vc"]
            V, T, K = (int(x) for x in h[0:6].view(np.int64))
            res = dict(counts=(V, T, K), labels=h[8:8 + V].copy(), vertex_point=h[8 + Vc:8 + Vc + V].copy())
            if self.copy_mesh:
                res["normals"] = bs["h_normals"][:V].numpy().copy()
                res["vertices"] = bs["h_vertices"][:V].numpy().copy()
                res["triangles"] = bs["h_triangles"][:T].numpy().copy()
            out.append(res)
            self.free_sets[r.sensor].append(bs)
        return out

    def discard(self, h):
        for r, bs in zip(h["reqs"], h["sets"]):
            self.free_sets[r.sensor].append(bs)

    def close(self):
        self.torch.cuda.synchronize()
        for c in self.ctxs:
            c.close()
