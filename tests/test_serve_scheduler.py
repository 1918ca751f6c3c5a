"""Continuous-batching scheduler on the CPU with a fake executor (no GPU):
admission by slots and memory budget, overlap, latency bookkeeping, results."""
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2005_02704_amd.serve import Request, Server, poisson_schedule


class FakeExecutor:
    """Completes a group `delay` seconds after submission; results from the oracle.
    Each request holds one buffer set of its sensor's pool while in flight, as the
    GPU executor's resident sets are held."""

    def __init__(self, n_slots, delay, sensors, sets_per_sensor=2):
        self.n_slots = n_slots
        self.delay = delay
        self.sensors = sensors
        self.submitted = []
        self.free_sets = [[object() for _ in range(sets_per_sensor)] for _ in sensors]
        self.sets_made = sets_per_sensor * len(sensors)

    def bytes_for(self, req):
        return 12 * req.n_points

    def _buffer_set(self, sensor):
        if self.free_sets[sensor]:
            return self.free_sets[sensor].pop()
        self.sets_made += 1
        return object()

    def submit(self, slot, reqs):
        self.submitted.append((slot, [r.rid for r in reqs]))
        return dict(t_ready=time.perf_counter() + self.delay, reqs=reqs,
                    sets=[self._buffer_set(r.sensor) for r in reqs])

    def poll(self, h):
        return time.perf_counter() >= h["t_ready"]

    def results(self, h):
        out = []
        for r, bs in zip(h["reqs"], h["sets"]):
            sen = self.sensors[r.sensor]
            res = oracle.mesh_segment(r.xyz, sen.n_rings, sen.n_azimuth, 1, sen.elevations())
            out.append(dict(labels=res.labels, counts=res.counts))
            self.free_sets[r.sensor].append(bs)
        return out

    def discard(self, h):
        for r, bs in zip(h["reqs"], h["sets"]):
            self.free_sets[r.sensor].append(bs)


@pytest.fixture(scope="module")
def frames():
    sens = [synth.Sensor.standard(16, 1024), synth.Sensor.standard(32, 1024)]
    fr = [[synth.make_frame(s, "street", 100 * q + k, sigma=0.01, dropout=0.1) for k in range(3)]
          for q, s in enumerate(sens)]
    return sens, fr


def _make(frames_):
    sens, fr = frames_

    def make(rid, sensor, payload, t):
        x = fr[sensor][payload].xyz
        return Request(rid, sensor, x, x.shape[0], t)
    return make


def test_all_served_with_overlap_and_batching(frames):
    sens, fr = frames
    ex = FakeExecutor(n_slots=2, delay=0.02, sensors=sens)
    srv = Server(ex, budget_bytes=10**9, max_batch=8)
    sched = poisson_schedule([200.0, 150.0], 0.3, seed=1, n_payloads=3)
    wall = srv.run_schedule(sched, _make(frames))
    st = srv.stats(wall)
    assert st["requests"] == len(sched)
    assert st["max_slots_in_flight"] == 2          # groups overlapped
    assert st["mean_batch"] > 1.0                  # arrivals during flight were batched
    assert all(r.t_done >= r.t_admit >= r.t_arrival for r in srv.done)
    assert st["p99_ms"] >= st["p50_ms"] >= 20.0 * 0.9
    # admission is FIFO across slots
    order = [rid for _, g in ex.submitted for rid in g]
    assert order == sorted(order)


def test_results_equal_alone(frames):
    sens, fr = frames
    ex = FakeExecutor(n_slots=3, delay=0.005, sensors=sens)
    srv = Server(ex, budget_bytes=10**9, max_batch=4)
    sched = poisson_schedule([300.0, 300.0], 0.1, seed=2, n_payloads=3)
    srv.run_schedule(sched, _make(frames))
    for r in srv.done:
        alone = oracle.mesh_segment(r.xyz, sens[r.sensor].n_rings, sens[r.sensor].n_azimuth, 1,
                                    sens[r.sensor].elevations())
        assert np.array_equal(r.result["labels"], alone.labels)


def test_memory_budget_limits_admission(frames):
    sens, fr = frames
    big = max(f.n_points for row in fr for f in row) * 12
    ex = FakeExecutor(n_slots=4, delay=0.01, sensors=sens)
    srv = Server(ex, budget_bytes=2 * big, max_batch=8)
    sched = [(0.0, q % 2, q % 3) for q in range(12)]
    srv.run_schedule(sched, _make(frames))
    assert srv.peak_in_use <= 2 * big
    assert len(srv.done) == 12
    # no group alone exceeds the budget, and the budget forced several groups
    sizes = {r.rid: 12 * r.n_points for r in srv.done}
    assert all(sum(sizes[i] for i in g) <= 2 * big for _, g in ex.submitted)
    assert len(ex.submitted) >= 4


def test_request_larger_than_budget_is_rejected(frames):
    sens, fr = frames
    ex = FakeExecutor(n_slots=1, delay=0.0, sensors=sens)
    srv = Server(ex, budget_bytes=10, max_batch=1)
    x = fr[0][0].xyz
    with pytest.raises(ValueError):
        srv.submit(Request(0, 0, x, x.shape[0], time.perf_counter()))


def test_poisson_schedule_rates():
    sched = poisson_schedule([10.0, 20.0], 60.0, seed=3, n_payloads=5)
    n0 = sum(1 for t, s, _ in sched if s == 0)
    n1 = sum(1 for t, s, _ in sched if s == 1)
    assert 480 < n0 < 720 and 1020 < n1 < 1380
    assert all(a[0] <= b[0] for a, b in zip(sched, sched[1:]))


class StuckExecutor(FakeExecutor):
    """Like FakeExecutor, but the groups that hold request `stuck` complete only
    when `release` is set: a device that stopped making progress."""

    def __init__(self, n_slots, delay, sensors, stuck):
        super().__init__(n_slots, delay, sensors)
        self.stuck = stuck
        self.release = False

    def poll(self, h):
        if any(r.rid == self.stuck for r in h["reqs"]) and not self.release:
            return False
        return super().poll(h)


def test_watchdog_fails_a_stuck_group_and_keeps_its_slot(frames):
    sens, fr = frames
    ex = StuckExecutor(n_slots=2, delay=0.005, sensors=sens, stuck=0)
    srv = Server(ex, budget_bytes=10**9, max_batch=1, timeout_s=0.05)
    make = _make(frames)
    for rid in range(6):
        srv.submit(make(rid, rid % 2, rid % 3, time.perf_counter()))
    t0 = time.perf_counter()
    while not srv.idle() and time.perf_counter() - t0 < 5.0:
        srv.step()
        time.sleep(1e-3)
    assert srv.idle()
    done = {r.rid: r for r in srv.done}
    assert sorted(done) == list(range(6))
    assert done[0].failed == "timeout" and done[0].result is None
    assert 0.05 <= done[0].latency < 1.0
    assert all(not done[k].failed and done[k].result is not None for k in range(1, 6))
    assert srv.failed == 1 and srv.stats(1.0)["failed"] == 1 and srv.stats(1.0)["requests"] == 5
    # the stuck group's slot was never reused: every other group ran on the other slot
    stuck_slot = done[0].slot
    assert all(done[k].slot != stuck_slot for k in range(1, 6))
    # its memory is released only when the device work completes
    assert srv.in_use == ex.bytes_for(done[0])
    assert sum(len(p) for p in ex.free_sets) == ex.sets_made - 1   # the stuck group holds one set
    ex.release = True
    srv.step()
    assert srv.in_use == 0 and not any(st.busy for st in srv.slots)
    assert len(srv.done) == 6   # the late completion adds no second result
    # the abandoned group's buffer set went back to its pool: every set made is free again
    assert sum(len(p) for p in ex.free_sets) == ex.sets_made
    # so later requests of that sensor reuse the pool instead of making new sets
    made = ex.sets_made
    for rid in range(6, 10):
        srv.submit(make(rid, 0, rid % 3, time.perf_counter()))
    while not srv.idle():
        srv.step()
        time.sleep(1e-3)
    assert ex.sets_made == made
