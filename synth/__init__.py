"""Seeded synthetic Lidar sweeps shared by tests, smoke and bench (input generation only)."""
from .scene import (ELEV_SPANS_DEG, Frame, Scene, Sensor, cast, frame_seed, make_frame,
                    make_scene, sample_frame)
from .workloads import WORKLOADS, batch_frames, batch_sensors, served_sensors, workload_frames

__all__ = ["ELEV_SPANS_DEG", "Frame", "Scene", "Sensor", "cast", "frame_seed", "make_frame",
           "make_scene", "sample_frame", "WORKLOADS", "workload_frames", "batch_sensors",
           "served_sensors", "batch_frames"]
