"""MI355X-native Lidar mesh + normal + segmentation path (HIP, gfx950).

The computation lives in liblidarseg.so (csrc/, C ABI in include/lidarseg.h);
this package is its thin Python binding plus the batching/serving loop around it.
"""
from .lidarseg import (EXPORTS, LAUNCH, STAGES, LIB_PATH, LIDAR_EDEVICE, LIDAR_EINVAL, LIDAR_ENOMEM,
                       LIDAR_LAUNCH_BATCHED, LIDAR_LAUNCH_GRAPH, LIDAR_LAUNCH_PLAIN, LIDAR_MAX_RINGS,
                       LIDAR_MAX_SCORE_RADIUS, LIDAR_N_STAGES, LIDAR_NOALLOC_MAX_FRAMES, LIDAR_NOALLOC_SCRATCH_BYTES, LIDAR_OK, LIDAR_PRED_COMPONENTS, LIDAR_PRED_COSINE, LidarContext,
                       LidarError, Outputs, SensorGeometry, lidar_mesh_segment, lidar_query_sizes, load_library,
                       make_params, precision_recall_f1)

__all__ = ["EXPORTS", "LAUNCH", "STAGES", "LIB_PATH", "LIDAR_EDEVICE", "LIDAR_EINVAL", "LIDAR_ENOMEM",
           "LIDAR_LAUNCH_BATCHED", "LIDAR_LAUNCH_GRAPH", "LIDAR_LAUNCH_PLAIN", "LIDAR_MAX_RINGS",
           "LIDAR_MAX_SCORE_RADIUS", "LIDAR_N_STAGES", "LIDAR_NOALLOC_MAX_FRAMES",
           "LIDAR_NOALLOC_SCRATCH_BYTES", "LIDAR_OK", "LIDAR_PRED_COMPONENTS", "LIDAR_PRED_COSINE", "LidarContext",
           "LidarError", "Outputs", "SensorGeometry", "lidar_mesh_segment",
           "lidar_query_sizes", "load_library", "make_params", "precision_recall_f1"]
