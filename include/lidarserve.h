/*
 * lidarserve.h -- C ABI of the served form of liblidarseg: a continuous-batching
 * server for sweeps from several sensors (part of liblidarseg.so).
 *
 * Requests are single sweeps (one spin P = {p(theta, phi, r)} of one sensor,
 * Section 2 of Mukherjee et al., PReMI 2019), each answered with its mesh
 * vertices' segment labels (Algorithm 1), vertex points and counts, computed by
 * lidar_mesh_segment.  A server thread inside the library admits waiting
 * requests first come first served into free slots -- one context and stream
 * each -- as groups of at most max_batch sweeps, while the device bytes that
 * admitted groups hold stay within the budget and each request gets a free
 * buffer set of its sensor; a group runs as one batched call (points copied in,
 * the chain, results copied out).  Requests arriving while groups run join the
 * next free slot, so groups overlap on the device.  Every buffer (device points
 * and outputs, pinned result blocks, each slot's workspace and captured graph)
 * is made when the server is created, so serving allocates nothing.
 *
 * Threads: submit, poll, result, release and stats may be called from any host
 * thread; each call is short (it takes the server's lock).
 * Return codes are those of lidarseg.h (LIDAR_OK or a negative LIDAR_E*).
 */
#ifndef LIDARSERVE_H
#define LIDARSERVE_H

#include <stdint.h>

#include "lidarseg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lidar_server lidar_server;

typedef struct {
    int32_t n_slots;          /* groups on the device at once, 1..16 */
    int32_t max_batch;        /* sweeps per group, 1..256 */
    int32_t launch;           /* LIDAR_LAUNCH_GRAPH, _BATCHED or _PLAIN */
    int32_t sets_per_sensor;  /* resident buffer sets of each sensor, >= 1: at most that many of a
                                 sensor's requests are in flight or hold unreleased results */
    uint64_t budget_bytes;    /* device bytes admitted groups may hold (per request: points,
                                 outputs and workspace share of its sensor); > 0 */
    double timeout_s;         /* watchdog per group, 0 = none: a group still running that long
                                 after launch fails its requests (LIDAR_SERVED_TIMED_OUT); its
                                 slot and sets stay held until the device work ends */
    int32_t copy_mesh;        /* 1: also copy vertices, normals and triangles back */
    int32_t tile_cells, tile_threads, grid;  /* launch shape of every slot (0 = library default) */
} lidar_server_opts_t;

/* Status of a finished request. */
#define LIDAR_SERVED_OK 2         /* results are held until lidar_server_release */
#define LIDAR_SERVED_TIMED_OUT 3  /* failed on the watchdog; no results */
#define LIDAR_SERVED_FAILED 4     /* its group could not be enqueued; no results */

typedef struct {
    int64_t id;
    int32_t sensor;
    int32_t status;           /* LIDAR_SERVED_* */
    int32_t slot, group_size; /* the slot and the size of the group it ran in */
    double t_arrival;         /* seconds on the server's clock: submission */
    double t_admit;           /* admission into a slot */
    double t_done;            /* the server saw the group's results on the host */
} lidar_served_t;

typedef struct {
    const int64_t* counts;        /* host [3]: V, T, K */
    const int32_t* labels;        /* host [V] */
    const int32_t* vertex_point;  /* host [V] */
    const float* vertices;        /* host [V][3] or NULL (copy_mesh) */
    const float* normals;         /* host [V][3] or NULL (copy_mesh) */
    const int32_t* triangles;     /* host [T][3] or NULL (copy_mesh) */
} lidar_server_result_t;

typedef struct {
    int64_t groups, admitted, timed_out, failed;
    uint64_t peak_bytes;          /* largest device bytes admitted groups held at once */
    int32_t max_slots_busy;       /* most groups on the device at once */
    uint64_t device_bytes;        /* device memory the server holds (sets and workspaces) */
} lidar_server_stats_t;

/* Creates a server on HIP device `device` for n_sensors sensors (geometry as
 * for lidar_mesh_segment; elevations are copied) with the given parameters,
 * makes every buffer, reserves each slot's workspace for the largest group
 * the budget admits, runs one empty group per slot (graph capture), then starts
 * the server thread. */
int lidar_server_create(int device, const lidar_sensor_t* sensors, int32_t n_sensors,
                        const lidar_params_t* params, const lidar_server_opts_t* opts,
                        lidar_server** out);
/* Stops the server thread after the device work in flight ends; frees everything. */
void lidar_server_destroy(lidar_server* srv);
/* Message of the calling thread's last failed server call (srv may be NULL). */
const char* lidar_server_last_error(const lidar_server* srv);

/* Queues one sweep of sensor `sensor`: xyz host [n_points][3] FP32 (pinned
 * memory lets the copy overlap), 0 <= n_points <= n_rings * n_azimuth.  The
 * points must stay valid until the request is reported finished, and, for a
 * request reported LIDAR_SERVED_TIMED_OUT (whose group may still be running),
 * until lidar_server_destroy.  Writes the request id. */
int lidar_server_submit(lidar_server* srv, int32_t sensor, const float* xyz, int64_t n_points,
                        int64_t* id);
/* Writes up to max finished requests (in completion order) and their number. */
int lidar_server_poll(lidar_server* srv, lidar_served_t* done, int32_t max, int32_t* n_done);
/* Host pointers to a served request's results, valid until it is released. */
int lidar_server_result(lidar_server* srv, int64_t id, lidar_server_result_t* out);
/* Returns a served request's buffer set to its pool. */
int lidar_server_release(lidar_server* srv, int64_t id);
int lidar_server_stats(lidar_server* srv, lidar_server_stats_t* out);
/* Seconds on the server's clock (the one lidar_served_t uses). */
double lidar_server_now(const lidar_server* srv);

/* Benchmark driver: submits n sweeps from the calling thread, request i at
 * t_offset[i] seconds after the call starts (offsets ascending), releases
 * each as it finishes, and returns when all have finished: latency_s[i] =
 * t_done - t_arrival, status[i] and group_size[i] per request (arrays of n,
 * may be NULL), wall_s = time from the call's start to the last finish.  It
 * consumes every finished request of the server while it runs. */
int lidar_server_replay(lidar_server* srv, int64_t n, const double* t_offset, const int32_t* sensor,
                        const float* const* xyz, const int64_t* n_points, double* latency_s,
                        int32_t* status, int32_t* group_size, double* wall_s);

#ifdef __cplusplus
}
#endif
#endif /* LIDARSERVE_H */
