"""The named synthetic workloads (sensor shapes, scene kinds, noise, dropouts).

Each stands in for the paper's BlenSor-simulated Velodyne scenes (Section 3), which
are not available: same kind of sensor lattice, primitive scenes, Gaussian range
noise and random dropouts, all seeded.
"""
from __future__ import annotations

import numpy as np

from .scene import Sensor, frame_seed, make_frame

# name -> dict(sensor=(H, W), kind, sigma, dropout, subsample(s), seed)
WORKLOADS = {
    # 16 rings (+15..-15 deg) x 1800 azimuth, ground + 3 boxes + 2 cylinders
    "c1_16x1800": dict(H=16, W=1800, kind="simple", sigma=0.02, dropout=0.05, s=(1,), seed=0),
    # 64 rings (+3..-25 deg) x 2048, street, s in {1, 2, 4}
    "c2_64x2048": dict(H=64, W=2048, kind="street", sigma=0.01, dropout=0.10, s=(1, 2, 4), seed=1),
    # 128 rings (+15..-25 deg) x 4096, dense urban on sloped ground, s = 2
    "c4_128x4096": dict(H=128, W=4096, kind="urban", sigma=0.01, dropout=0.10, s=(2,), seed=4),
    # the paper's own shape: 32 rings x 1800 firings (0.2 deg), intervals 5/10/15
    "paper_32x1800": dict(H=32, W=1800, kind="street", sigma=0.01, dropout=0.0, s=(5, 10, 15), seed=7),
}

BATCH_RINGS = (16, 32, 64, 128)
BATCH_WIDTHS = (1024, 2048, 4096)


def workload_frames(name: str, n_frames: int = 1, base_seed: int | None = None):
    """Frames of a single-sensor workload; frame f uses seed frame_seed(base, f)."""
    w = WORKLOADS[name]
    base = w["seed"] if base_seed is None else base_seed
    sensor = Sensor.standard(w["H"], w["W"]) if w["H"] in (16, 32, 64, 128) else None
    return [make_frame(sensor, w["kind"], frame_seed(base, f), sigma=w["sigma"], dropout=w["dropout"])
            for f in range(n_frames)]


def batch_sensors(n_frames: int, seed: int):
    """Uneven batch: rings uniform over {16,32,64,128}, widths over {1024,2048,4096}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    hs = rng.choice(BATCH_RINGS, size=n_frames)
    ws = rng.choice(BATCH_WIDTHS, size=n_frames)
    return [Sensor.standard(int(h), int(w)) for h, w in zip(hs, ws)]


def batch_frames(n_frames: int, seed: int, *, sigma=0.01, dropout=0.10, kind="street"):
    """The batched workload: n_frames street sweeps of uneven sensor shapes, per-frame seeds."""
    sensors = batch_sensors(n_frames, seed)
    return [make_frame(s, kind, frame_seed(seed, f), sigma=sigma, dropout=dropout)
            for f, s in enumerate(sensors)]


def served_sensors(n_sensors: int = 8):
    """Sensor q: rings (16,32,64,128)[q % 4], width (1024,2048,4096)[q % 3], rate 10 + 10 q / 7 Hz."""
    out = []
    for q in range(n_sensors):
        out.append((Sensor.standard(BATCH_RINGS[q % 4], BATCH_WIDTHS[q % 3]),
                    10.0 + 10.0 * q / max(1, n_sensors - 1)))
    return out
