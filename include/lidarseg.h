/*
 * lidarseg.h -- C ABI of the MI355X (gfx950) Lidar mesh-and-segment library.
 *
 * One spinning-Lidar sweep P = {p(theta, phi, r)} (Mukherjee et al., PReMI 2019,
 * Section 2, opening paragraph) is turned into
 *   - the vertices of its sub-sampled (ring x azimuth) lattice,
 *   - the mesh triangles joining lattice neighbours      (Section 2, Mesh Construction),
 *   - one normal per vertex                              (Section 2, Normal Estimation),
 *   - one surface label per vertex                       (Section 2, Algorithm 1).
 *
 * Conventions shared by every entry point
 *   - All data pointers named "device" are HIP device memory owned by the caller;
 *     they must stay valid until the work enqueued on `stream` has finished.
 *   - Calls are asynchronous: they validate arguments on the host, enqueue work on
 *     `stream` (a hipStream_t; NULL = the default stream) and return.
 *   - Return codes: LIDAR_OK (0) or a negative LIDAR_E* code; the message of the
 *     last failure is available from lidar_ctx_last_error().  Argument errors are
 *     reported before anything is enqueued.
 *   - A context is used by one host thread at a time; contexts are independent and
 *     may run concurrently on different streams.  The calls made on one context
 *     are ordered on the device even when they name different streams: they share
 *     the context's workspace, so a call on another stream than the context's
 *     previous call first makes its stream wait (hipStreamWaitEvent) for the end
 *     of that call.  Work of other streams and contexts is not waited for.
 *
 * Lattice conventions (see also the readings in the repository's design notes)
 *   - Ring i = 0 is the topmost laser, counting downwards; elevations are given
 *     strictly descending.  Azimuth phi = atan2(y, x) (anticlockwise about +z);
 *     firing j has phi_j = az0 + j * 2*pi / W.  A point belongs to the ring of
 *     nearest elevation (tie: lower i), or to the ring the sensor reported for it
 *     (lidar_frame_t.ring_ids), and to firing round((phi - az0)/dphi) mod W
 *     (round half away from zero); both decided in FP64.
 *   - Sub-sampling keeps firings j = 0 (mod s); sampled column k = j / s, W' = W / s.
 *   - A point is used iff its coordinates are finite and
 *     r_min^2 <= x^2 + y^2 + z^2 <= r_max^2 (FP64).  Two points in one cell: the
 *     smaller float(r^2) wins, then the lower input index.
 *   - Vertices are the occupied cells, numbered in firing order: column-major,
 *     (k, i) lexicographic.  Labels 1..K are numbered by each segment's first
 *     vertex in that order.
 */
#ifndef LIDARSEG_H
#define LIDARSEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LIDAR_OK 0
#define LIDAR_EINVAL (-1)   /* bad argument; nothing was enqueued */
#define LIDAR_ENOMEM (-2)   /* device workspace could not be allocated, or would exceed the
                               context's limit (lidar_ctx_set_workspace_limit) */
#define LIDAR_EDEVICE (-3)  /* a HIP runtime call failed */

#define LIDAR_MAX_RINGS 128

/* Launch forms of lidar_mesh_segment. */
#define LIDAR_LAUNCH_PLAIN 0    /* each frame on its own: one kernel chain per frame */
#define LIDAR_LAUNCH_BATCHED 1  /* all frames together: one grid-stride launch per stage */
#define LIDAR_LAUNCH_GRAPH 2    /* the batched chain replayed from a captured hipGraph */

typedef struct lidar_ctx lidar_ctx;

/* Sensor geometry (Section 2, Mesh Construction: rings theta_0..theta_n from the
 * top, firings phi_0..phi_m from the first shot of the spin). */
typedef struct {
    int32_t n_rings;         /* H, 1..LIDAR_MAX_RINGS */
    int32_t n_azimuth;       /* W, firings per spin, >= 1 */
    int32_t subsample;       /* s >= 1, W % s == 0 (the paper's sampling interval) */
    int32_t wrap;            /* 1: join column W'-1 to column 0 (closed cylinder); 0: open */
    const double* elev_rad;  /* host, H ring elevations in radians, strictly descending */
    double az0_rad;          /* azimuth of firing 0, in [-2 pi, 2 pi] */
} lidar_sensor_t;

/* One sweep. */
typedef struct {
    const lidar_sensor_t* sensor;  /* host */
    const float* xyz;              /* device, [n_points][3] FP32, any order */
    int64_t n_points;              /* 0 .. 2^31-1 */
    const float* normals_in;       /* device [>= V][3] or NULL.  When given, the normal
                                      stage is skipped and these per-vertex normals
                                      (zero vector = no normal) are labelled instead;
                                      row v is vertex v's normal, and the buffer must
                                      hold at least this frame's vertex count V of
                                      rows (max_vertices of lidar_query_sizes always
                                      suffices; the kernels read rows 0 .. V-1). */
    const int32_t* truth_ids;      /* device [n_points] or NULL: ground-truth surface id
                                      of every input point, read only for the edge
                                      scores (lidar_result_t.edge_counts) */
    const uint8_t* ring_ids;       /* device [n_points] or NULL: the ring (laser) each
                                      point was fired by, as the sensor reports it; it
                                      replaces the nearest-elevation decision, and a
                                      point whose ring is >= n_rings is not used */
} lidar_frame_t;

/* Similarity tests of lidar_params_t.predicate. */
#define LIDAR_PRED_COMPONENTS 0  /* Algorithm 1: every normal component differs by < I, J, K */
#define LIDAR_PRED_COSINE 1      /* n_p . n_q > cos_min (dot product of the FP32 normals,
                                    summed in FP64 as (x x' + y y') + z z') */

/* Parameters (Section 2, Mesh Construction "within range of the Lidar";
 * Algorithm 1 thresholds I, J, K, which Section 3 sets to 0.2 each; Section 2,
 * Segmentation, last paragraph: optional removal of segments with too few
 * points). */
typedef struct {
    double r_min, r_max;  /* valid range window in metres, 0 <= r_min <= r_max */
    double thr[3];        /* I, J, K > 0: a neighbour joins when every component of
                             the normal differs by strictly less (exact FP64 difference
                             of the FP32 normals) */
    int32_t predicate;    /* LIDAR_PRED_COMPONENTS (default) or LIDAR_PRED_COSINE */
    int32_t min_segment;  /* >= 2: labels carried by fewer vertices become 0 (the count
                             K is unchanged); 0 or 1: keep every segment */
    double cos_min;       /* LIDAR_PRED_COSINE threshold, in [-1, 1) */
    int32_t score_radius; /* edge scores: dilation radius R in lattice steps,
                             0..LIDAR_MAX_SCORE_RADIUS */
} lidar_params_t;

#define LIDAR_MAX_SCORE_RADIUS 8

/* Caller-owned outputs of one frame, sized by lidar_query_sizes().  Written
 * compactly from index 0; counts tells how many entries are valid. */
typedef struct {
    float* vertices;        /* device [V][3]: the kept input points, bit-exact */
    float* normals;         /* device [V][3]: unit normals, zero vector = no normal */
    int32_t* labels;        /* device [V]: 1..K */
    int32_t* triangles;     /* device [T][3]: vertex indices, each oriented so that
                               (v1-v0) x (v2-v0) points away from the sensor */
    int32_t* vertex_point;  /* device [V] or NULL: input index of each vertex */
    int64_t* counts;        /* device [3]: V, T, K */
    int32_t* point_labels;  /* device [n_points] or NULL: every input point's label
                               (Section 2, Segmentation: the points the sub-sampling
                               skipped take the label of the nearest vertex of their
                               ring along the sweep, by firing distance -- around the
                               cylinder when it is closed -- the earlier firing on a
                               tie); 0 for a point that is not used or whose ring has
                               no vertex */
    int64_t* edge_counts;   /* device [4] or NULL: edge scores of the labels against
                               the frame's truth_ids (Section 3 scores segmentations
                               by their dilated edge points: precision, recall, F1).
                               A vertex is a segment edge when a mesh join reaches a
                               vertex of another label (after segment removal), a
                               truth edge when one reaches a vertex of another truth
                               id.  Written: {segment edges, truth edges, segment
                               edges with a truth edge within R rings and R columns
                               (around the cylinder when closed), truth edges with a
                               segment edge that near}.  precision = [2] / [0],
                               recall = [3] / [1].  Needs truth_ids. */
} lidar_result_t;

/* Create a context on HIP device `device`.  The context owns its device
 * workspace (grown on demand) and any captured graph. */
int lidar_ctx_create(int device, lidar_ctx** out);
void lidar_ctx_destroy(lidar_ctx* ctx);
/* Message of the last failed call on this context ("" if none).  Owned by ctx. */
const char* lidar_ctx_last_error(const lidar_ctx* ctx);
/* Message of the last failure outside any context (creation, size queries). */
const char* lidar_last_error(void);

/* Output capacities for one frame of this sensor: V <= H*W', T <= 2*(H-1)*W'.
 * A lattice may hold at most 2^29 cells. */
int lidar_query_sizes(const lidar_sensor_t* sensor, int64_t* max_vertices,
                      int64_t* max_triangles);

/* Bin, sub-sample, mesh, estimate normals and label n_frames sweeps
 * (Section 2 in full; Algorithm 1 is computed as the connected components of
 * the similar-join graph, which is the partition it produces).
 * launch: LIDAR_LAUNCH_PLAIN, _BATCHED or _GRAPH.  results has n_frames entries. */
int lidar_mesh_segment(lidar_ctx* ctx, const lidar_frame_t* frames, int32_t n_frames,
                       const lidar_params_t* params, lidar_result_t* results,
                       void* stream, int32_t launch);

/* Section 2 up to Normal Estimation only (binning, sub-sampling, mesh, normals):
 * the same kernels as lidar_mesh_segment without the labelling stages, for
 * callers (and tests) that want the mesh and its normals alone.  Arguments as
 * for lidar_mesh_segment, except: only r_min and r_max of params are read;
 * results[f].labels may be NULL and is not written; counts[2] (K) is written
 * as 0; frames[f].normals_in, results[f].point_labels and results[f].edge_counts
 * must be NULL (LIDAR_EINVAL otherwise). */
int lidar_mesh_normals(lidar_ctx* ctx, const lidar_frame_t* frames, int32_t n_frames,
                       const lidar_params_t* params, lidar_result_t* results,
                       void* stream, int32_t launch);

/* Algorithm 1 on normals the caller gives (the labelling stages on the
 * lattice and mesh of each sweep): lidar_mesh_segment with
 * frames[f].normals_in required for every frame that has points (LIDAR_EINVAL
 * otherwise).  The given normals are copied to results[f].normals. */
int lidar_label_grid(lidar_ctx* ctx, const lidar_frame_t* frames, int32_t n_frames,
                     const lidar_params_t* params, lidar_result_t* results,
                     void* stream, int32_t launch);

/* For callers that cannot allocate memory -- code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation: lidar_mesh_segment
 * (same arguments, same kernels, same outputs bit for bit) that calls no
 * hipMalloc, hipFree, hipHostMalloc or other allocating routine.  Differences:
 *   - the workspace and the descriptor table live in one fixed array of
 *     LIDAR_NOALLOC_SCRATCH_BYTES of device memory per GPU, which the GPU holds
 *     from the library's first use on it until the process ends (the pinned host
 *     staging of the table is made by lidar_ctx_create).  A call that needs more
 *     (roughly 12 bytes per lattice cell of the batch, 12 more per cell when
 *     point labels, segment removal or edge scores are asked for, 4 per input
 *     point with point labels) returns LIDAR_ENOMEM before anything is
 *     enqueued; the message gives the bytes needed;
 *   - launch is LIDAR_LAUNCH_PLAIN or LIDAR_LAUNCH_BATCHED (LIDAR_EINVAL for
 *     LIDAR_LAUNCH_GRAPH, which would create a graph), and n_frames is at most
 *     LIDAR_NOALLOC_MAX_FRAMES;
 *   - every call on one GPU uses that GPU's one array, which keeps the last
 *     call's contents (each call first resets the state the kernels expect).
 *     Calls made on one context are ordered as for every entry point; calls of
 *     different contexts on one GPU that overlap on the device race, so the
 *     caller orders them (one stream, or events);
 *   - per-stage timing (lidar_ctx_set_profiling) does not record these calls,
 *     and the context's own workspace (lidar_ctx_workspace_bytes) is not used. */
#define LIDAR_NOALLOC_SCRATCH_BYTES (64ull << 20)
#define LIDAR_NOALLOC_MAX_FRAMES 64
int lidar_mesh_segment_noalloc(lidar_ctx* ctx, const lidar_frame_t* frames, int32_t n_frames,
                               const lidar_params_t* params, lidar_result_t* results,
                               void* stream, int32_t launch);

/* Device workspace.  A context grows its workspace when a call needs more
 * (by half as much again as asked for, to reallocate rarely) and keeps it until
 * it is destroyed.  With a limit set (max_bytes > 0; 0 = none), a call whose
 * batch would take the workspace above it returns LIDAR_ENOMEM before anything
 * is enqueued (the growth slack is dropped first); memory already held is not
 * released by a lower limit.  lidar_ctx_workspace_bytes writes the device
 * bytes the context holds now (pinned host staging not included). */
int lidar_ctx_set_workspace_limit(lidar_ctx* ctx, uint64_t max_bytes);
int lidar_ctx_workspace_bytes(const lidar_ctx* ctx, uint64_t* held_bytes);

/* Launch shape of every later call on this context: workgroups per grid-stride
 * stage (0 = automatic: 4 per compute unit), the largest tile in lattice cells
 * and the threads of a tile workgroup.  Supported tile shapes (cells, threads):
 * (512, 256), (1024, 256), (2048, 256), (1024, 512), (2048, 512); 0 selects
 * 1024 cells or 256 threads.  Results do not depend on the shape.  A change
 * of shape drops the captured graph, after waiting for this context's earlier
 * graph replays to finish (a host wait). */
int lidar_ctx_set_tuning(lidar_ctx* ctx, int32_t grid_workgroups, int32_t tile_cells, int32_t tile_threads);

/* Workgroups of one stage (index in the order of the stage list below) in
 * batched and graph launches of later calls, in place of its share of the
 * grid set by lidar_ctx_set_tuning; 0 restores that share.  Results do not
 * depend on it.  A change waits and drops the graph as lidar_ctx_set_tuning. */
int lidar_ctx_set_stage_grid(lidar_ctx* ctx, int32_t stage, int32_t workgroups);

/* Per-stage timing of plain and batched launches (not of graph replays), with
 * HIP events recorded on the launch stream around each kernel of the chain.
 * Stages, in order: bin, count (vertices, triangles and occupancy per tile),
 * geom (numbering, mesh triangles, normals), cc (similar joins, local
 * segments), merge (segments across tiles), compress (pointer jumping on the
 * merged segments), flatten (segment roots), scan (rank bases of the roots),
 * label, post (segment removal and point labels; zero time when neither is
 * asked for), score (edge scores; zero time unless asked for).  In
 * lidar_mesh_normals calls the labelling stages take zero time and flatten is
 * the reset of the key grid.  Enabling costs one event per kernel. */
#define LIDAR_N_STAGES 11
int lidar_ctx_set_profiling(lidar_ctx* ctx, int32_t enable);
/* Waits for the profiled calls, then writes the summed milliseconds and the
 * number of timed launches of each stage (arrays of LIDAR_N_STAGES; launches
 * may be NULL) and resets the accumulators. */
int lidar_ctx_stage_times(lidar_ctx* ctx, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* LIDARSEG_H */
