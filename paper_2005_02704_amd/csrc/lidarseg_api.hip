// Host side of liblidarseg: argument validation, workspace planning, descriptor
// tables, launch forms (plain per-frame chains, one batched chain, or a captured
// hipGraph of the batched chain).  The C ABI is declared in include/lidarseg.h.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lidarseg.h"
#include "lidarseg_internal.h"

using namespace lidarseg;

namespace {

thread_local std::string g_last_error;

constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Pinned staging of the descriptor table of lidar_mesh_segment_noalloc: the
// larger of the batched table and the plain tables of LIDAR_NOALLOC_MAX_FRAMES
// frames of LIDAR_MAX_RINGS rings each.
constexpr size_t NOALLOC_TABLE_BATCHED =
    align_up(sizeof(BatchHeader) + sizeof(FrameDesc) * LIDAR_NOALLOC_MAX_FRAMES, 8) +
    8 * (size_t)LIDAR_NOALLOC_MAX_FRAMES * LIDAR_MAX_RINGS;
constexpr size_t NOALLOC_TABLE_PLAIN =
    LIDAR_NOALLOC_MAX_FRAMES * align_up(sizeof(BatchHeader) + sizeof(FrameDesc) + 8 * (size_t)LIDAR_MAX_RINGS, 256);
constexpr size_t NOALLOC_TABLE_BYTES =
    NOALLOC_TABLE_BATCHED > NOALLOC_TABLE_PLAIN ? NOALLOC_TABLE_BATCHED : NOALLOC_TABLE_PLAIN;

// The workspace of lidar_mesh_segment_noalloc: one fixed array per GPU, which
// each GPU holds from the library's first use on it until the process ends.
// On the host this name only stands for the symbol: host code never passes it
// to a kernel or a copy, but the device address looked up for each device.
static __device__ __align__(256) unsigned char scratch[LIDAR_NOALLOC_SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
bool g_scratch_looked_up[SCRATCH_MAX_DEVICES] = {};
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
hipError_t g_scratch_err[SCRATCH_MAX_DEVICES] = {};

// Looks up the device address of `scratch` on `device`, which must be the
// current device, once per device (every GPU holds its own copy of the array at
// its own address).
void scratch_lookup(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_looked_up[device]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();  // the failure is reported by the entry point
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_scratch_looked_up[device] = true;
}

// The device address of `scratch` on `device` (looked up by lidar_ctx_create),
// or nullptr with the lookup's error.
void* scratch_address(int device, hipError_t* err) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) { *err = hipErrorInvalidDevice; return nullptr; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *err = g_scratch_looked_up[device] ? g_scratch_err[device] : hipErrorNotInitialized;
    return g_scratch_ptr[device];
}

}  // namespace

struct lidar_ctx {
    int device = 0;
    int cu_count = 256;
    std::string err;

    // device workspace
    uint64_t* keys = nullptr;
    int32_t* forest = nullptr;    // same capacity as keys
    int64_t keys_cap = 0;
    int32_t* tile_buf = nullptr;  // 3 int32 arrays of tiles_cap: vertices, triangles, vertex base per tile
    uint64_t* occ = nullptr;      // OCC_WORDS per tile
    int64_t tiles_cap = 0;
    uint64_t* rootbits = nullptr; // VITEM_WORDS per labelling item
    uint32_t* wprefix = nullptr;  // VITEM_WORDS per labelling item
    int32_t* vitem_roots = nullptr;  // one per labelling item
    int64_t vitems_cap = 0;
    int2* border = nullptr;
    int64_t border_cap = 0;
    int32_t* pcell = nullptr;     // per input point record (point labels)
    int64_t pcell_cap = 0;
    int32_t* cvid = nullptr;      // per cell vertex id (point labels, edge scores)
    int32_t* segsize = nullptr;   // per label size (segment removal)
    int32_t* vtruth = nullptr;    // per vertex truth id (edge scores)
    int64_t aux_cells_cap = 0;    // capacity of cvid, segsize and vtruth
    char* d_table = nullptr;      // descriptor tables + elevations
    char* h_table[2] = {nullptr, nullptr};  // pinned staging of d_table, used alternately
    char* na_table[2] = {nullptr, nullptr}; // pinned staging of lidar_mesh_segment_noalloc's table
                                            // (NOALLOC_TABLE_BYTES each, made with the context)
    size_t table_cap = 0;
    hipEvent_t done[2] = {nullptr, nullptr};  // end of the call that last used h_table[b]
    bool pending[2] = {false, false};
    int flip = 0;
    hipStream_t last_stream = nullptr;  // stream of the previous call (its end is done[flip ^ 1])

    // captured batched chain
    // Two instantiations of the same captured chain, launched alternately, so a
    // launch never has to wait for the previous launch of the same executable.
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    int graph_next = 0;
    bool graph_valid = false;
    size_t graph_table_bytes = 0;
    int graph_tile_cells = 0;
    int graph_tile_threads = 0;
    int graph_grid = 0;
    bool graph_post = false;
    bool graph_score = false;
    bool graph_mesh_only = false;

    uint64_t ws_limit = 0;        // device workspace bytes the context may hold (0 = no limit)

    // Device bytes of the workspace at the given capacities.
    static uint64_t ws_bytes(int64_t keys_n, int64_t tiles_n, int64_t vitems_n, int64_t pcell_n, int64_t aux_n,
                             int64_t border_n, size_t table_n) {
        return (uint64_t)keys_n * (sizeof(uint64_t) + sizeof(int32_t)) +
               (uint64_t)tiles_n * (3 * sizeof(int32_t) + OCC_WORDS * sizeof(uint64_t)) +
               (uint64_t)vitems_n * (VITEM_WORDS * (sizeof(uint64_t) + sizeof(uint32_t)) + sizeof(int32_t)) +
               (uint64_t)pcell_n * sizeof(int32_t) +
               (uint64_t)aux_n * 3 * sizeof(int32_t) + (uint64_t)border_n * sizeof(int2) + (uint64_t)table_n;
    }
    uint64_t held_bytes() const {
        return ws_bytes(keys_cap, tiles_cap, vitems_cap, pcell_cap, aux_cells_cap, border_cap, table_cap);
    }

    // tuning
    int grid_wg = 0;      // 0 = automatic
    int stage_grid[N_STAGES] = {0};  // per stage workgroups of batched and graph launches, 0 = from grid_wg
    int tile_cells = 1024;
    int tile_threads = 256;

    // per-stage timing
    bool profiling = false;
    std::vector<std::vector<hipEvent_t>> prof_sets;  // one set of N_STAGES+1 events per chain
    std::vector<hipEvent_t> prof_free;
    double prof_ms[N_STAGES] = {0};
    int64_t prof_n[N_STAGES] = {0};

    hipEvent_t* new_event_set() {
        std::vector<hipEvent_t> set(N_STAGES + 1);
        for (auto& ev : set) {
            if (!prof_free.empty()) {
                ev = prof_free.back();
                prof_free.pop_back();
            } else if (hipEventCreate(&ev) != hipSuccess) {
                return nullptr;
            }
        }
        prof_sets.push_back(std::move(set));
        return prof_sets.back().data();
    }

    int fail(int code, const std::string& msg) {
        err = msg;
        g_last_error = msg;
        return code;
    }
    int hip_fail(hipError_t e, const char* what) {
        return fail(LIDAR_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
    Workspace workspace() const {
        Workspace ws;
        ws.keys = keys;
        ws.forest = forest;
        ws.tile_v = tile_buf;
        ws.tile_t = tile_buf + tiles_cap;
        ws.tile_vbase = tile_buf + 2 * tiles_cap;
        ws.occ = occ;
        ws.rootbits = rootbits;
        ws.wprefix = wprefix;
        ws.vitem_roots = vitem_roots;
        ws.border = border;
        ws.pcell = pcell;
        ws.cvid = cvid;
        ws.segsize = segsize;
        ws.vtruth = vtruth;
        ws.elev = reinterpret_cast<const double*>(d_table);
        return ws;
    }
    void drop_graph() {
        for (auto& ge : graph_exec) {
            if (ge) (void)hipGraphExecDestroy(ge);
            ge = nullptr;
        }
        if (graph) (void)hipGraphDestroy(graph);
        graph = nullptr;
        graph_valid = false;
    }
    int wait_buffer(int b) {
        if (pending[b]) {
            hipError_t e = hipEventSynchronize(done[b]);
            if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
            pending[b] = false;
        }
        return LIDAR_OK;
    }
    int wait_idle() {
        int rc = wait_buffer(0);
        return rc ? rc : wait_buffer(1);
    }
};

namespace {

struct FramePlan {
    int H, W, s, Wp, wrap, TW, n_tiles, n_pblk, n_vitem;
    int64_t cells, border_slots;
};

int validate_sensor(const lidar_sensor_t* sen, std::string& msg) {
    if (!sen) { msg = "sensor is NULL"; return LIDAR_EINVAL; }
    const int H = sen->n_rings, W = sen->n_azimuth, s = sen->subsample;
    if (H < 1 || H > LIDAR_MAX_RINGS) { msg = "n_rings must be in [1, 128]"; return LIDAR_EINVAL; }
    if (W < 1) { msg = "n_azimuth must be >= 1"; return LIDAR_EINVAL; }
    if (s < 1 || W % s != 0) { msg = "subsample must be >= 1 and divide n_azimuth"; return LIDAR_EINVAL; }
    if (sen->wrap != 0 && sen->wrap != 1) { msg = "wrap must be 0 or 1"; return LIDAR_EINVAL; }
    if (sen->wrap && W / s < 3) { msg = "a closed cylinder needs at least 3 sampled columns"; return LIDAR_EINVAL; }
    if ((int64_t)H * (W / s) > MAX_CELLS) { msg = "lattice too large (at most 2^29 cells)"; return LIDAR_EINVAL; }
    if (!sen->elev_rad) { msg = "elev_rad is NULL"; return LIDAR_EINVAL; }
    for (int i = 0; i < H; ++i) {
        if (!std::isfinite(sen->elev_rad[i])) { msg = "elevations must be finite"; return LIDAR_EINVAL; }
        if (i > 0 && !(sen->elev_rad[i] < sen->elev_rad[i - 1])) {
            msg = "elevations must be strictly descending (ring 0 = top)";
            return LIDAR_EINVAL;
        }
    }
    if (!(std::fabs(sen->az0_rad) <= 2.0 * M_PI)) { msg = "az0_rad must lie in [-2 pi, 2 pi]"; return LIDAR_EINVAL; }
    return LIDAR_OK;
}

}  // namespace

extern "C" {

const char* lidar_last_error(void) { return g_last_error.c_str(); }

const char* lidar_ctx_last_error(const lidar_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int lidar_query_sizes(const lidar_sensor_t* sensor, int64_t* max_vertices, int64_t* max_triangles) {
    std::string msg;
    int rc = validate_sensor(sensor, msg);
    if (rc) { g_last_error = msg; return rc; }
    const int64_t Wp = sensor->n_azimuth / sensor->subsample;
    if (max_vertices) *max_vertices = (int64_t)sensor->n_rings * Wp;
    if (max_triangles) *max_triangles = 2 * (int64_t)(sensor->n_rings - 1) * Wp;
    return LIDAR_OK;
}

int lidar_ctx_create(int device, lidar_ctx** out) {
    if (!out) { g_last_error = "out is NULL"; return LIDAR_EINVAL; }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device < 0 || device >= n) {
        g_last_error = "no such HIP device";
        return LIDAR_EINVAL;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) { g_last_error = hipGetErrorString(e); return LIDAR_EDEVICE; }
    lidar_ctx* c = new lidar_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->cu_count = prop.multiProcessorCount;
    for (int b = 0; b < 2; ++b) {
        e = hipEventCreateWithFlags(&c->done[b], hipEventDisableTiming);
        if (e != hipSuccess) { g_last_error = hipGetErrorString(e); lidar_ctx_destroy(c); return LIDAR_EDEVICE; }
        e = hipHostMalloc(&c->na_table[b], NOALLOC_TABLE_BYTES, hipHostMallocDefault);
        if (e != hipSuccess) {
            c->na_table[b] = nullptr;
            g_last_error = "cannot allocate the pinned table staging";
            lidar_ctx_destroy(c);
            return LIDAR_ENOMEM;
        }
    }
    // the no-allocation entry point's scratch address on this device (once per device)
    scratch_lookup(device);
    *out = c;
    return LIDAR_OK;
}

void lidar_ctx_destroy(lidar_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    c->wait_idle();
    c->drop_graph();
    for (auto& set : c->prof_sets)
        for (auto ev : set) (void)hipEventDestroy(ev);
    for (auto ev : c->prof_free) (void)hipEventDestroy(ev);
    if (c->keys) (void)hipFree(c->keys);
    if (c->forest) (void)hipFree(c->forest);
    if (c->tile_buf) (void)hipFree(c->tile_buf);
    if (c->occ) (void)hipFree(c->occ);
    if (c->rootbits) (void)hipFree(c->rootbits);
    if (c->wprefix) (void)hipFree(c->wprefix);
    if (c->vitem_roots) (void)hipFree(c->vitem_roots);
    if (c->border) (void)hipFree(c->border);
    if (c->pcell) (void)hipFree(c->pcell);
    if (c->cvid) (void)hipFree(c->cvid);
    if (c->segsize) (void)hipFree(c->segsize);
    if (c->vtruth) (void)hipFree(c->vtruth);
    if (c->d_table) (void)hipFree(c->d_table);
    for (int b = 0; b < 2; ++b) {
        if (c->h_table[b]) (void)hipHostFree(c->h_table[b]);
        if (c->na_table[b]) (void)hipHostFree(c->na_table[b]);
        if (c->done[b]) (void)hipEventDestroy(c->done[b]);
    }
    delete c;
}

int lidar_ctx_set_tuning(lidar_ctx* c, int32_t grid_workgroups, int32_t tile_cells, int32_t tile_threads) {
    if (!c) return LIDAR_EINVAL;
    if (grid_workgroups < 0) return c->fail(LIDAR_EINVAL, "grid_workgroups must be >= 0");
    const int cells = tile_cells ? tile_cells : 1024;
    const int threads = tile_threads ? tile_threads : 256;
    if (!tile_shape_supported(cells, threads))
        return c->fail(LIDAR_EINVAL, "unsupported tile shape (cells, threads): use (512|1024|2048, 256) "
                                     "or (1024|2048, 512)");
    if (c->grid_wg == grid_workgroups && c->tile_cells == cells && c->tile_threads == threads) return LIDAR_OK;
    // a replay of the captured chain may still run: wait for this context's
    // earlier calls before the graph is destroyed
    const int rc = c->wait_idle();
    if (rc) return rc;
    c->grid_wg = grid_workgroups;
    c->tile_cells = cells;
    c->tile_threads = threads;
    c->drop_graph();
    return LIDAR_OK;
}

int lidar_ctx_set_stage_grid(lidar_ctx* c, int32_t stage, int32_t workgroups) {
    if (!c) { g_last_error = "ctx is NULL"; return LIDAR_EINVAL; }
    if (stage < 0 || stage >= N_STAGES) return c->fail(LIDAR_EINVAL, "stage must lie in [0, LIDAR_N_STAGES)");
    if (workgroups < 0) return c->fail(LIDAR_EINVAL, "workgroups must be >= 0");
    if (c->stage_grid[stage] == workgroups) return LIDAR_OK;
    const int rc = c->wait_idle();  // as in lidar_ctx_set_tuning
    if (rc) return rc;
    c->stage_grid[stage] = workgroups;
    c->drop_graph();
    return LIDAR_OK;
}

int lidar_ctx_set_workspace_limit(lidar_ctx* c, uint64_t max_bytes) {
    if (!c) { g_last_error = "ctx is NULL"; return LIDAR_EINVAL; }
    c->ws_limit = max_bytes;
    return LIDAR_OK;
}

int lidar_ctx_workspace_bytes(const lidar_ctx* c, uint64_t* held_bytes) {
    if (!c || !held_bytes) { g_last_error = "ctx or held_bytes is NULL"; return LIDAR_EINVAL; }
    *held_bytes = c->held_bytes();
    return LIDAR_OK;
}

int lidar_ctx_set_profiling(lidar_ctx* c, int32_t enable) {
    if (!c) return LIDAR_EINVAL;
    c->profiling = enable != 0;
    return LIDAR_OK;
}

int lidar_ctx_stage_times(lidar_ctx* c, double* total_ms, int64_t* launches) {
    if (!c || !total_ms) return LIDAR_EINVAL;
    for (auto& set : c->prof_sets) {
        hipError_t e = hipEventSynchronize(set[N_STAGES]);
        if (e != hipSuccess) return c->hip_fail(e, "hipEventSynchronize");
        for (int k = 0; k < N_STAGES; ++k) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, set[k], set[k + 1]);
            if (e != hipSuccess) return c->hip_fail(e, "hipEventElapsedTime");
            c->prof_ms[k] += ms;
            c->prof_n[k] += 1;
        }
        for (auto ev : set) c->prof_free.push_back(ev);
    }
    c->prof_sets.clear();
    for (int k = 0; k < N_STAGES; ++k) {
        total_ms[k] = c->prof_ms[k];
        if (launches) launches[k] = c->prof_n[k];
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    return LIDAR_OK;
}

}  // extern "C"

namespace {

enum CallMode { CALL_SEGMENT = 0, CALL_MESH_ONLY = 1, CALL_LABEL_GRID = 2 };

// One roctx range per library call (named by entry point), visible to
// rocprofv3 --marker-trace; without a tool attached the calls do nothing.
struct CallRange {
    explicit CallRange(const char* name) { roctxRangePushA(name); }
    ~CallRange() { roctxRangePop(); }
};

// What one call needs: sums over its frames (batched and graph forms), or the
// largest frame (plain form: the frames run one after another on shared
// workspace offsets).
struct CallTotals {
    int64_t cells = 0, border_slots = 0, elev_total = 0, tiles = 0, pblk = 0, vitems = 0;
    int64_t labelled_points = 0;  // point records (frames asking for point labels)
    bool any_point_labels = false, any_score = false, prune = false, post = false, aux = false;
    size_t table_bytes = 0;       // descriptor table (header, descriptors, elevations)
};

// Host-side validation of every argument and the plan of each frame; nothing
// is enqueued.  plan has n_frames entries.
int plan_call(lidar_ctx* c, const lidar_frame_t* frames, int32_t n_frames, const lidar_params_t* params,
              const lidar_result_t* results, int32_t launch, CallMode mode, FramePlan* plan, CallTotals& tot) {
    const bool mesh_only = mode == CALL_MESH_ONLY;
    if (n_frames < 1 || !frames || !results) return c->fail(LIDAR_EINVAL, "need n_frames >= 1 frames and results");
    if (!params) return c->fail(LIDAR_EINVAL, "params is NULL");
    if (launch != LIDAR_LAUNCH_PLAIN && launch != LIDAR_LAUNCH_BATCHED && launch != LIDAR_LAUNCH_GRAPH)
        return c->fail(LIDAR_EINVAL, "unknown launch form");
    const double rmin = params->r_min, rmax = params->r_max;
    if (!(std::isfinite(rmin) && std::isfinite(rmax) && rmin >= 0.0 && rmin <= rmax))
        return c->fail(LIDAR_EINVAL, "need finite 0 <= r_min <= r_max");
    if (!mesh_only) {  // the similarity test and segment floor matter only to the labelling stages
        for (int q = 0; q < 3; ++q)
            if (!(std::isfinite(params->thr[q]) && params->thr[q] > 0.0))
                return c->fail(LIDAR_EINVAL, "thresholds must be finite and > 0");
        if (params->predicate != LIDAR_PRED_COMPONENTS && params->predicate != LIDAR_PRED_COSINE)
            return c->fail(LIDAR_EINVAL, "unknown predicate");
        if (params->predicate == LIDAR_PRED_COSINE &&
            !(std::isfinite(params->cos_min) && params->cos_min >= -1.0 && params->cos_min < 1.0))
            return c->fail(LIDAR_EINVAL, "cos_min must lie in [-1, 1)");
        if (params->min_segment < 0) return c->fail(LIDAR_EINVAL, "min_segment must be >= 0");
    }

    tot = CallTotals();
    int64_t max_points_f = 0, max_cells = 0, max_tiles_f = 0, max_vitem_f = 0, max_border_f = 0;
    for (int f = 0; f < n_frames; ++f) {
        const lidar_frame_t& fr = frames[f];
        std::string msg;
        int rc = validate_sensor(fr.sensor, msg);
        if (rc) return c->fail(rc, "frame " + std::to_string(f) + ": " + msg);
        if (mesh_only && (fr.normals_in || results[f].point_labels || results[f].edge_counts))
            return c->fail(LIDAR_EINVAL, "frame " + std::to_string(f) +
                                             ": lidar_mesh_normals estimates normals and labels nothing "
                                             "(normals_in, point_labels and edge_counts must be NULL)");
        if (mode == CALL_LABEL_GRID && fr.n_points > 0 && !fr.normals_in)
            return c->fail(LIDAR_EINVAL, "frame " + std::to_string(f) + ": lidar_label_grid needs normals_in");
        if (fr.n_points < 0 || fr.n_points > INT32_MAX)
            return c->fail(LIDAR_EINVAL, "frame " + std::to_string(f) + ": n_points out of range");
        if (results[f].point_labels) {
            if ((int64_t)fr.sensor->n_rings * fr.sensor->n_azimuth > INT32_MAX)
                return c->fail(LIDAR_EINVAL, "frame " + std::to_string(f) +
                                                 ": point labels need n_rings * n_azimuth below 2^31");
            tot.any_point_labels = true;
            tot.labelled_points += fr.n_points;
            max_points_f = std::max<int64_t>(max_points_f, fr.n_points);
        }
        if (fr.n_points > 0 && !fr.xyz)
            return c->fail(LIDAR_EINVAL, "frame " + std::to_string(f) + ": xyz is NULL");
        if (results[f].edge_counts) {
            if (fr.n_points > 0 && !fr.truth_ids)
                return c->fail(LIDAR_EINVAL, "frame " + std::to_string(f) + ": edge scores need truth_ids");
            if (params->score_radius < 0 || params->score_radius > LIDAR_MAX_SCORE_RADIUS)
                return c->fail(LIDAR_EINVAL, "score_radius must lie in [0, LIDAR_MAX_SCORE_RADIUS]");
            tot.any_score = true;
        }
        const lidar_result_t& r = results[f];
        if (!r.vertices || !r.normals || (!r.labels && !mesh_only) || !r.triangles || !r.counts)
            return c->fail(LIDAR_EINVAL, "result " + std::to_string(f) + ": a required output is NULL");
        FramePlan& p = plan[f];
        p.H = fr.sensor->n_rings;
        p.W = fr.sensor->n_azimuth;
        p.s = fr.sensor->subsample;
        p.Wp = p.W / p.s;
        p.wrap = fr.sensor->wrap;
        p.TW = tile_width(p.H, c->tile_cells);
        p.n_tiles = (p.Wp + p.TW - 1) / p.TW;
        p.n_pblk = (int)((fr.n_points + POINT_BLOCK - 1) / POINT_BLOCK);
        p.cells = (int64_t)p.H * p.Wp;
        p.n_vitem = (int)((p.cells + VITEM - 1) / VITEM);
        p.border_slots = (int64_t)p.n_tiles * 2 * p.H;
        tot.cells += p.cells;
        tot.border_slots += p.border_slots;
        tot.elev_total += p.H;
        tot.tiles += p.n_tiles;
        tot.pblk += p.n_pblk;
        tot.vitems += p.n_vitem;
        max_cells = std::max(max_cells, p.cells);
        max_tiles_f = std::max<int64_t>(max_tiles_f, p.n_tiles);
        max_vitem_f = std::max<int64_t>(max_vitem_f, p.n_vitem);
        max_border_f = std::max(max_border_f, p.border_slots);
    }
    if (tot.tiles > INT32_MAX || tot.pblk > INT32_MAX || tot.cells > MAX_BATCH_CELLS ||
        tot.border_slots > INT32_MAX)
        return c->fail(LIDAR_EINVAL, "batch too large (at most 2^31 - 1024 lattice cells in one call)");
    tot.prune = !mesh_only && params->min_segment > 1;
    tot.post = tot.prune || tot.any_point_labels;
    tot.aux = tot.any_point_labels || tot.prune || tot.any_score;
    // table bytes: batched = one header, all descs, elevations; plain = one
    // (header, desc, elevations) group per frame.
    if (launch == LIDAR_LAUNCH_PLAIN) {
        for (int f = 0; f < n_frames; ++f)
            tot.table_bytes += align_up(sizeof(BatchHeader) + sizeof(FrameDesc) + 8 * (size_t)plan[f].H, 256);
        // plain launches run the frames one after another on shared workspace offsets
        tot.labelled_points = max_points_f;
        tot.cells = max_cells;
        tot.tiles = max_tiles_f;
        tot.vitems = max_vitem_f;
        tot.border_slots = max_border_f;
    } else {
        tot.table_bytes = align_up(sizeof(BatchHeader) + sizeof(FrameDesc) * n_frames, 8) + 8 * (size_t)tot.elev_total;
    }
    return LIDAR_OK;
}

// Makes `stream` wait (on the device) for the context's previous call when
// that call was enqueued on another stream: calls on one context share its
// workspace and device table.
int order_after_previous_call(lidar_ctx* c, hipStream_t stream) {
    if (c->pending[c->flip ^ 1] && stream != c->last_stream) {
        const hipError_t e = hipStreamWaitEvent(stream, c->done[c->flip ^ 1], 0);
        if (e != hipSuccess) return c->hip_fail(e, "hipStreamWaitEvent");
    }
    return LIDAR_OK;
}

// Fills the descriptor table in the pinned host buffer htab (header,
// descriptors and elevations; for plain launches one group per frame at
// group_off[f]), copies it to d_table on `stream` and enqueues the kernels:
// one chain per frame (plain) or one chain over the batch (batched).  The
// graph form is launched by the caller from the same table.
int enqueue_table_and_chains(lidar_ctx* c, const lidar_frame_t* frames, int32_t n_frames,
                             const lidar_params_t* params, const lidar_result_t* results, const FramePlan* plan,
                             const CallTotals& tot, int32_t launch, bool mesh_only, hipStream_t stream,
                             const Workspace& ws, char* d_table, char* htab, bool profile) {
    const size_t desc_bytes = sizeof(FrameDesc);
    std::memset(htab, 0, tot.table_bytes);
    const double rmin = params->r_min, rmax = params->r_max;
    auto fill_desc = [&](FrameDesc& d, int f, int64_t cell_off, int64_t border_off, int64_t pt_off, int tile_off,
                         int pblk_off, int vitem_off, int elev_off) {
        const lidar_frame_t& fr = frames[f];
        const lidar_result_t& r = results[f];
        const FramePlan& p = plan[f];
        d.xyz = fr.xyz;
        d.normals_in = fr.normals_in;
        d.vertices = r.vertices;
        d.normals = r.normals;
        d.labels = r.labels;
        d.tris = r.triangles;
        d.vpoint = r.vertex_point;
        d.counts = r.counts;
        d.n_points = fr.n_points;
        d.cell_off = cell_off;
        d.border_off = border_off;
        d.pt_off = pt_off;
        d.point_labels = r.point_labels;
        d.truth = r.edge_counts ? fr.truth_ids : nullptr;
        d.rings = fr.ring_ids;
        d.scores = r.edge_counts;
        d.score_r = params->score_radius;
        d.pred = params->predicate;
        d.min_seg = mesh_only ? 0 : params->min_segment;
        d.cos_min = params->cos_min;
        d.H = p.H; d.W = p.W; d.s = p.s; d.Wp = p.Wp; d.wrap = p.wrap; d.TW = p.TW;
        d.n_tiles = p.n_tiles; d.tile_off = tile_off;
        d.n_pblk = p.n_pblk; d.pblk_off = pblk_off;
        d.n_vitem = p.n_vitem; d.vitem_off = vitem_off;
        d.elev_off = elev_off;
        d.az0 = fr.sensor->az0_rad;
        d.dphi = 2.0 * M_PI / (double)p.W;
        d.rmin2 = rmin * rmin;
        d.rmax2 = rmax * rmax;
        d.thr[0] = params->thr[0]; d.thr[1] = params->thr[1]; d.thr[2] = params->thr[2];
        std::memcpy(htab + 8 * (size_t)elev_off, fr.sensor->elev_rad, 8 * (size_t)p.H);
    };
    hipError_t e;
    if (launch == LIDAR_LAUNCH_PLAIN) {
        size_t off = 0;
        for (int f = 0; f < n_frames; ++f) {
            BatchHeader* h = reinterpret_cast<BatchHeader*>(htab + off);
            h->n_frames = 1;
            h->total_tiles = plan[f].n_tiles;
            h->total_pblk = plan[f].n_pblk;
            h->total_vitems = plan[f].n_vitem;
            h->total_border = (int)plan[f].border_slots;
            h->post = (tot.prune || results[f].point_labels) ? 1 : 0;
            const size_t elev_byte = off + sizeof(BatchHeader) + desc_bytes;
            // frames run one after another on the stream, so they share workspace offsets
            fill_desc(*h->frames(), f, 0, 0, 0, 0, 0, 0, (int)(elev_byte / 8));
            off += align_up(sizeof(BatchHeader) + desc_bytes + 8 * (size_t)plan[f].H, 256);
        }
        e = hipMemcpyAsync(d_table, htab, tot.table_bytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync");
        off = 0;
        for (int f = 0; f < n_frames; ++f) {
            LaunchCfg cfg;
            cfg.tile_cells = c->tile_cells;
            cfg.tile_threads = c->tile_threads;
            cfg.max_tiles = plan[f].n_tiles;
            cfg.max_pblk = plan[f].n_pblk;
            cfg.max_vitems = plan[f].n_vitem;
            cfg.max_border = (int)plan[f].border_slots;
            cfg.max_frames = 1;
            cfg.post = tot.prune || results[f].point_labels;
            cfg.score = results[f].edge_counts != nullptr;
            cfg.mesh_only = mesh_only;
            cfg.grid = std::max(std::max(plan[f].n_tiles, plan[f].n_pblk), plan[f].n_vitem);
            hipEvent_t* ev = profile ? c->new_event_set() : nullptr;
            e = launch_chain(reinterpret_cast<const BatchHeader*>(d_table + off), ws, cfg, stream, ev);
            if (e != hipSuccess) return c->hip_fail(e, "kernel launch");
            off += align_up(sizeof(BatchHeader) + desc_bytes + 8 * (size_t)plan[f].H, 256);
        }
        return LIDAR_OK;
    }
    BatchHeader* h = reinterpret_cast<BatchHeader*>(htab);
    h->n_frames = n_frames;
    h->total_tiles = (int)tot.tiles;
    h->total_pblk = (int)tot.pblk;
    h->total_vitems = (int)tot.vitems;
    h->total_border = (int)tot.border_slots;
    h->post = tot.post ? 1 : 0;
    FrameDesc* d = h->frames();
    const size_t elev_base = align_up(sizeof(BatchHeader) + desc_bytes * n_frames, 8) / 8;
    int64_t cell_off = 0, border_off = 0, pt_off = 0;
    int tile_off = 0, pblk_off = 0, vitem_off = 0, elev_off = (int)elev_base;
    for (int f = 0; f < n_frames; ++f) {
        fill_desc(d[f], f, cell_off, border_off, pt_off, tile_off, pblk_off, vitem_off, elev_off);
        cell_off += plan[f].cells;
        border_off += plan[f].border_slots;
        if (results[f].point_labels) pt_off += frames[f].n_points;
        tile_off += plan[f].n_tiles;
        pblk_off += plan[f].n_pblk;
        vitem_off += plan[f].n_vitem;
        elev_off += plan[f].H;
    }
    // the device table is read only by this call's kernels, which run after
    // this copy in stream order; the next call's copy follows them likewise
    e = hipMemcpyAsync(d_table, htab, tot.table_bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync");
    if (launch == LIDAR_LAUNCH_BATCHED) {
        LaunchCfg cfg;
        cfg.tile_cells = c->tile_cells;
        cfg.tile_threads = c->tile_threads;
        cfg.max_tiles = (int)tot.tiles;
        cfg.max_pblk = (int)tot.pblk;
        cfg.max_vitems = (int)tot.vitems;
        cfg.max_border = (int)tot.border_slots;
        cfg.max_frames = n_frames;
        cfg.post = tot.post;
        cfg.score = tot.any_score;
        cfg.mesh_only = mesh_only;
        cfg.grid = c->grid_wg > 0 ? c->grid_wg : 4 * c->cu_count;
        std::copy(c->stage_grid, c->stage_grid + N_STAGES, cfg.stage_grid);
        hipEvent_t* ev = profile ? c->new_event_set() : nullptr;
        e = launch_chain(reinterpret_cast<const BatchHeader*>(d_table), ws, cfg, stream, ev);
        if (e != hipSuccess) return c->hip_fail(e, "kernel launch");
    }
    return LIDAR_OK;
}

// Records the end of the call that used pinned table `buf` on `stream`.
int finish_call(lidar_ctx* c, int buf, hipStream_t stream) {
    const hipError_t e = hipEventRecord(c->done[buf], stream);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventRecord");
    c->pending[buf] = true;
    c->last_stream = stream;
    c->flip ^= 1;
    c->err.clear();
    return LIDAR_OK;
}

// Grows the context's workspace (and descriptor-table staging) to hold a call
// with these totals; the graph is dropped when anything is reallocated.
// Growth waits for the context's earlier calls and for the device.
int ensure_capacity(lidar_ctx* c, const CallTotals& tot, hipStream_t stream) {
    const int64_t cells = tot.cells, tiles = tot.tiles, vitems = tot.vitems, border_slots = tot.border_slots;
    const int64_t labelled_points = tot.labelled_points;
    const bool any_point_labels = tot.any_point_labels;
    const size_t table_bytes = tot.table_bytes;
    hipError_t e;
    const bool aux_needed = tot.aux;
    const bool grow = cells > c->keys_cap || tiles > c->tiles_cap || vitems > c->vitems_cap ||
                      border_slots > c->border_cap || table_bytes > c->table_cap ||
                      (any_point_labels && labelled_points > c->pcell_cap) ||
                      (aux_needed && cells > c->aux_cells_cap);
    // new capacities: half as much again as asked for, so that a slowly
    // growing stream of batches reallocates rarely, unless that slack would
    // break the context's workspace limit
    int64_t n_keys = c->keys_cap, n_tiles = c->tiles_cap, n_vitems = c->vitems_cap, n_pcell = c->pcell_cap,
            n_aux = c->aux_cells_cap, n_border = c->border_cap;
    size_t n_table = c->table_cap;
    for (int exact = 0; grow && exact < 2; ++exact) {
        auto cap = [&](int64_t need, int64_t have) {
            return need <= have ? have : exact ? need : std::max<int64_t>(need, have * 3 / 2);
        };
        n_keys = cap(cells, c->keys_cap);
        n_tiles = cap(tiles, c->tiles_cap);
        n_vitems = cap(vitems, c->vitems_cap);
        n_pcell = any_point_labels ? cap(labelled_points, c->pcell_cap) : c->pcell_cap;
        n_aux = aux_needed ? cap(cells, c->aux_cells_cap) : c->aux_cells_cap;
        n_border = cap(border_slots, c->border_cap);
        n_table = table_bytes <= c->table_cap ? c->table_cap
                  : align_up(exact ? table_bytes : std::max(table_bytes, c->table_cap * 3 / 2), 4096);
        const uint64_t want = lidar_ctx::ws_bytes(n_keys, n_tiles, n_vitems, n_pcell, n_aux, n_border, n_table);
        if (!c->ws_limit || want <= c->ws_limit) break;
        if (exact)
            return c->fail(LIDAR_ENOMEM, "the batch needs " + std::to_string(want) +
                                             " bytes of device workspace, above the context's limit of " +
                                             std::to_string(c->ws_limit));
    }
    if (grow) {
        int rc = c->wait_idle();
        if (rc) return rc;
        (void)hipDeviceSynchronize();
        c->drop_graph();
        if (cells > c->keys_cap) {
            if (c->keys) (void)hipFree(c->keys);
            if (c->forest) (void)hipFree(c->forest);
            c->keys = nullptr;
            c->forest = nullptr;
            const int64_t cap = n_keys;
            if (hipMalloc(&c->keys, sizeof(uint64_t) * cap) != hipSuccess ||
                hipMalloc(&c->forest, sizeof(int32_t) * cap) != hipSuccess) {
                c->keys_cap = 0;
                return c->fail(LIDAR_ENOMEM, "cannot allocate the key grid");
            }
            // every chain resets the cells it used, so this fill happens once
            e = fill_keys_empty(c->keys, cap, stream);
            if (e != hipSuccess) return c->hip_fail(e, "key grid fill");
            c->keys_cap = cap;
        }
        if (tiles > c->tiles_cap) {
            if (c->tile_buf) (void)hipFree(c->tile_buf);
            if (c->occ) (void)hipFree(c->occ);
            c->tile_buf = nullptr;
            c->occ = nullptr;
            const int64_t cap = n_tiles;
            if (hipMalloc(&c->tile_buf, sizeof(int32_t) * 3 * cap) != hipSuccess ||
                hipMalloc(&c->occ, sizeof(uint64_t) * OCC_WORDS * cap) != hipSuccess) {
                c->tiles_cap = 0;
                return c->fail(LIDAR_ENOMEM, "cannot allocate tile arrays");
            }
            c->tiles_cap = cap;
        }
        if (vitems > c->vitems_cap) {
            if (c->rootbits) (void)hipFree(c->rootbits);
            if (c->wprefix) (void)hipFree(c->wprefix);
            if (c->vitem_roots) (void)hipFree(c->vitem_roots);
            c->rootbits = nullptr;
            c->wprefix = nullptr;
            c->vitem_roots = nullptr;
            const int64_t cap = n_vitems;
            if (hipMalloc(&c->rootbits, sizeof(uint64_t) * VITEM_WORDS * cap) != hipSuccess ||
                hipMalloc(&c->wprefix, sizeof(uint32_t) * VITEM_WORDS * cap) != hipSuccess ||
                hipMalloc(&c->vitem_roots, sizeof(int32_t) * cap) != hipSuccess) {
                c->vitems_cap = 0;
                return c->fail(LIDAR_ENOMEM, "cannot allocate labelling arrays");
            }
            c->vitems_cap = cap;
        }
        if (any_point_labels && labelled_points > c->pcell_cap) {
            if (c->pcell) (void)hipFree(c->pcell);
            c->pcell = nullptr;
            const int64_t cap = n_pcell;
            if (hipMalloc(&c->pcell, sizeof(int32_t) * std::max<int64_t>(cap, 1)) != hipSuccess) {
                c->pcell_cap = 0;
                return c->fail(LIDAR_ENOMEM, "cannot allocate point records");
            }
            c->pcell_cap = cap;
        }
        if (aux_needed && cells > c->aux_cells_cap) {
            if (c->cvid) (void)hipFree(c->cvid);
            if (c->segsize) (void)hipFree(c->segsize);
            if (c->vtruth) (void)hipFree(c->vtruth);
            c->cvid = nullptr;
            c->segsize = nullptr;
            c->vtruth = nullptr;
            const int64_t cap = n_aux;
            if (hipMalloc(&c->cvid, sizeof(int32_t) * cap) != hipSuccess ||
                hipMalloc(&c->segsize, sizeof(int32_t) * cap) != hipSuccess ||
                hipMalloc(&c->vtruth, sizeof(int32_t) * cap) != hipSuccess) {
                c->aux_cells_cap = 0;
                return c->fail(LIDAR_ENOMEM, "cannot allocate per-cell label arrays");
            }
            c->aux_cells_cap = cap;
        }
        if (border_slots > c->border_cap) {
            if (c->border) (void)hipFree(c->border);
            c->border = nullptr;
            const int64_t cap = n_border;
            if (hipMalloc(&c->border, sizeof(int2) * cap) != hipSuccess) {
                c->border_cap = 0;
                return c->fail(LIDAR_ENOMEM, "cannot allocate border slots");
            }
            c->border_cap = cap;
        }
        if (table_bytes > c->table_cap) {
            if (c->d_table) (void)hipFree(c->d_table);
            c->d_table = nullptr;
            for (int b = 0; b < 2; ++b) {
                if (c->h_table[b]) (void)hipHostFree(c->h_table[b]);
                c->h_table[b] = nullptr;
            }
            const size_t cap = n_table;
            if (hipMalloc(&c->d_table, cap) != hipSuccess ||
                hipHostMalloc(&c->h_table[0], cap, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc(&c->h_table[1], cap, hipHostMallocDefault) != hipSuccess) {
                c->table_cap = 0;
                return c->fail(LIDAR_ENOMEM, "cannot allocate descriptor tables");
            }
            c->table_cap = cap;
        }
    }

    return LIDAR_OK;
}

int mesh_call(lidar_ctx* c, const lidar_frame_t* frames, int32_t n_frames, const lidar_params_t* params,
              lidar_result_t* results, void* stream_, int32_t launch, CallMode mode) {
    if (!c) { g_last_error = "ctx is NULL"; return LIDAR_EINVAL; }
    const CallRange range(mode == CALL_MESH_ONLY ? "lidar_mesh_normals"
                          : mode == CALL_LABEL_GRID ? "lidar_label_grid" : "lidar_mesh_segment");
    const bool mesh_only = mode == CALL_MESH_ONLY;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);

    // ---- plan ----
    std::vector<FramePlan> plan(n_frames > 0 ? n_frames : 0);
    CallTotals tot;
    {
        const int rc = plan_call(c, frames, n_frames, params, results, launch, mode, plan.data(), tot);
        if (rc) return rc;
    }
    const int64_t cells = tot.cells, tiles = tot.tiles, vitems = tot.vitems, border_slots = tot.border_slots;
    const int64_t labelled_points = tot.labelled_points;
    const bool any_point_labels = tot.any_point_labels, any_score = tot.any_score, post = tot.post;
    const size_t table_bytes = tot.table_bytes;

    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return c->hip_fail(e, "hipSetDevice");

    // ---- capacity ----
    {
        const int rc = ensure_capacity(c, tot, stream);
        if (rc) return rc;
    }

    // ---- calls on one context are ordered ----
    // Every call reuses the context's workspace and device table, so a call on
    // another stream than the previous one first waits, on the device, for
    // that call's end.  (Growth above already waited for it on the host.)
    {
        const int rc = order_after_previous_call(c, stream);
        if (rc) return rc;
    }

    // ---- fill a pinned table (after the call that used it last has finished) ----
    const int buf = c->flip;
    {
        int rc = c->wait_buffer(buf);
        if (rc) return rc;
    }
    const Workspace ws = c->workspace();
    {
        const int rc = enqueue_table_and_chains(c, frames, n_frames, params, results, plan.data(), tot, launch,
                                                mesh_only, stream, ws, c->d_table, c->h_table[buf], c->profiling);
        if (rc) return rc;
    }
    if (launch == LIDAR_LAUNCH_GRAPH) {
        const int auto_grid = c->grid_wg > 0 ? c->grid_wg : 4 * c->cu_count;
        // The captured chain uses fixed grid-stride grids and reads the batch
        // from the device table, so it serves every batch that fits the workspace.
        if (!c->graph_valid || c->graph_table_bytes != c->table_cap || c->graph_tile_cells != c->tile_cells ||
            c->graph_tile_threads != c->tile_threads || c->graph_grid != auto_grid || c->graph_post != post ||
            c->graph_score != any_score || c->graph_mesh_only != mesh_only) {
            // a replay of the old graph may still run: wait for this
            // context's earlier calls before destroying it
            int rc = c->wait_idle();
            if (rc) return rc;
            c->drop_graph();
            hipStream_t cap_stream;
            e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return c->hip_fail(e, "hipStreamCreate");
            e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) { (void)hipStreamDestroy(cap_stream); return c->hip_fail(e, "hipStreamBeginCapture"); }
            LaunchCfg cfg;
            cfg.tile_cells = c->tile_cells;
            cfg.tile_threads = c->tile_threads;
            cfg.max_tiles = (int)std::min<int64_t>(c->tiles_cap, INT32_MAX);
            cfg.max_pblk = INT32_MAX;
            cfg.max_vitems = (int)std::min<int64_t>(c->vitems_cap, INT32_MAX);
            cfg.max_border = (int)std::min<int64_t>(c->border_cap, INT32_MAX);
            cfg.max_frames = INT32_MAX;
            cfg.post = post;
            cfg.score = any_score;
            cfg.mesh_only = mesh_only;
            cfg.grid = auto_grid;
            std::copy(c->stage_grid, c->stage_grid + N_STAGES, cfg.stage_grid);
            hipError_t e2 = launch_chain(reinterpret_cast<const BatchHeader*>(c->d_table), ws, cfg, cap_stream);
            e = hipStreamEndCapture(cap_stream, &c->graph);
            (void)hipStreamDestroy(cap_stream);
            if (e2 != hipSuccess) return c->hip_fail(e2, "capture launch");
            if (e != hipSuccess) return c->hip_fail(e, "hipStreamEndCapture");
            for (auto& ge : c->graph_exec) {
                e = hipGraphInstantiate(&ge, c->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) { c->drop_graph(); return c->hip_fail(e, "hipGraphInstantiate"); }
            }
            c->graph_valid = true;
            c->graph_table_bytes = c->table_cap;
            c->graph_tile_cells = c->tile_cells;
            c->graph_tile_threads = c->tile_threads;
            c->graph_grid = auto_grid;
            c->graph_post = post;
            c->graph_score = any_score;
            c->graph_mesh_only = mesh_only;
        }
        e = hipGraphLaunch(c->graph_exec[c->graph_next], stream);
        c->graph_next ^= 1;
        if (e != hipSuccess) return c->hip_fail(e, "hipGraphLaunch");
    }
    return finish_call(c, buf, stream);
}

// lidar_mesh_segment with the workspace and the device table carved out of the
// per-device scratch array; allocates nothing.
int mesh_call_noalloc(lidar_ctx* c, const lidar_frame_t* frames, int32_t n_frames, const lidar_params_t* params,
                      lidar_result_t* results, void* stream_, int32_t launch) {
    if (!c) { g_last_error = "ctx is NULL"; return LIDAR_EINVAL; }
    const CallRange range("lidar_mesh_segment_noalloc");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    if (launch == LIDAR_LAUNCH_GRAPH)
        return c->fail(LIDAR_EINVAL, "lidar_mesh_segment_noalloc launches plain or batched chains only "
                                     "(a graph would have to be created)");
    if (n_frames > LIDAR_NOALLOC_MAX_FRAMES)
        return c->fail(LIDAR_EINVAL, "lidar_mesh_segment_noalloc takes at most LIDAR_NOALLOC_MAX_FRAMES (" +
                                         std::to_string(LIDAR_NOALLOC_MAX_FRAMES) + ") frames");
    FramePlan plan[LIDAR_NOALLOC_MAX_FRAMES];
    CallTotals tot;
    {
        const int rc = plan_call(c, frames, n_frames, params, results, launch, CALL_SEGMENT, plan, tot);
        if (rc) return rc;
    }
    // the workspace's arrays, one after another at 256-byte boundaries
    size_t used = 0;
    auto take = [&](size_t bytes) {
        const size_t at = used;
        used = align_up(used + bytes, 256);
        return at;
    };
    const size_t o_keys = take(sizeof(uint64_t) * tot.cells);
    const size_t o_forest = take(sizeof(int32_t) * tot.cells);
    const size_t o_tiles = take(3 * sizeof(int32_t) * tot.tiles);
    const size_t o_occ = take(OCC_WORDS * sizeof(uint64_t) * tot.tiles);
    const size_t o_rootbits = take(VITEM_WORDS * sizeof(uint64_t) * tot.vitems);
    const size_t o_wprefix = take(VITEM_WORDS * sizeof(uint32_t) * tot.vitems);
    const size_t o_vroots = take(sizeof(int32_t) * tot.vitems);
    const size_t o_border = take(sizeof(int2) * tot.border_slots);
    const size_t o_pcell = take(tot.any_point_labels ? sizeof(int32_t) * tot.labelled_points : 0);
    const size_t o_cvid = take(tot.aux ? sizeof(int32_t) * tot.cells : 0);
    const size_t o_segsize = take(tot.aux ? sizeof(int32_t) * tot.cells : 0);
    const size_t o_vtruth = take(tot.aux ? sizeof(int32_t) * tot.cells : 0);
    const size_t o_table = take(tot.table_bytes);
    if (used > LIDAR_NOALLOC_SCRATCH_BYTES)
        return c->fail(LIDAR_ENOMEM, "the call needs " + std::to_string(used) +
                                         " bytes of workspace, above the no-allocation scratch of " +
                                         std::to_string((unsigned long long)LIDAR_NOALLOC_SCRATCH_BYTES) + " bytes");
    if (tot.table_bytes > NOALLOC_TABLE_BYTES)  // cannot happen within the frame and ring limits
        return c->fail(LIDAR_EINVAL, "descriptor table larger than its pinned staging");

    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return c->hip_fail(e, "hipSetDevice");
    char* const base = static_cast<char*>(scratch_address(c->device, &e));
    if (!base) return c->hip_fail(e, "scratch address of this device");

    {
        const int rc = order_after_previous_call(c, stream);
        if (rc) return rc;
    }
    const int buf = c->flip;
    {
        const int rc = c->wait_buffer(buf);
        if (rc) return rc;
    }
    Workspace ws;
    ws.keys = reinterpret_cast<uint64_t*>(base + o_keys);
    ws.forest = reinterpret_cast<int32_t*>(base + o_forest);
    ws.tile_v = reinterpret_cast<int32_t*>(base + o_tiles);
    ws.tile_t = ws.tile_v + tot.tiles;
    ws.tile_vbase = ws.tile_v + 2 * tot.tiles;
    ws.occ = reinterpret_cast<uint64_t*>(base + o_occ);
    ws.rootbits = reinterpret_cast<uint64_t*>(base + o_rootbits);
    ws.wprefix = reinterpret_cast<uint32_t*>(base + o_wprefix);
    ws.vitem_roots = reinterpret_cast<int32_t*>(base + o_vroots);
    ws.border = reinterpret_cast<int2*>(base + o_border);
    ws.pcell = tot.any_point_labels ? reinterpret_cast<int32_t*>(base + o_pcell) : nullptr;
    ws.cvid = tot.aux ? reinterpret_cast<int32_t*>(base + o_cvid) : nullptr;
    ws.segsize = tot.aux ? reinterpret_cast<int32_t*>(base + o_segsize) : nullptr;
    ws.vtruth = tot.aux ? reinterpret_cast<int32_t*>(base + o_vtruth) : nullptr;
    char* const d_table = base + o_table;
    ws.elev = reinterpret_cast<const double*>(d_table);
    // the array keeps whatever the last call on this GPU left in it: the key
    // grid, the only state the chain expects, starts empty (a fill kernel)
    e = fill_keys_empty(ws.keys, tot.cells, stream);
    if (e != hipSuccess) return c->hip_fail(e, "key grid fill");
    {
        const int rc = enqueue_table_and_chains(c, frames, n_frames, params, results, plan, tot, launch, false,
                                                stream, ws, d_table, c->na_table[buf], false);
        if (rc) return rc;
    }
    return finish_call(c, buf, stream);
}

}  // namespace

int lidarseg::ctx_reserve(lidar_ctx* c, const lidar_sensor_t* sensors, int32_t n_sensors, int32_t max_frames,
                          uint64_t budget, const uint64_t* bytes_per_sensor, bool plain, hipStream_t stream) {
    if (!c || !sensors || n_sensors < 1 || max_frames < 1 || !bytes_per_sensor) return LIDAR_EINVAL;
    // Each total is at most max_frames times its largest per-sweep value, and at
    // most the budget times its largest value per byte of a sweep.
    constexpr int NQ = 5;  // cells, tiles, labelling items, border slots, rings
    int64_t most[NQ] = {0, 0, 0, 0, 0};
    double per_byte[NQ] = {0, 0, 0, 0, 0};
    for (int s = 0; s < n_sensors; ++s) {
        std::string msg;
        const int rc = validate_sensor(&sensors[s], msg);
        if (rc) return c->fail(rc, "sensor " + std::to_string(s) + ": " + msg);
        const int H = sensors[s].n_rings, Wp = sensors[s].n_azimuth / sensors[s].subsample;
        const int TW = tile_width(H, c->tile_cells);
        const int64_t cells = (int64_t)H * Wp, tiles = (Wp + TW - 1) / TW;
        const int64_t q[NQ] = {cells, tiles, (cells + VITEM - 1) / VITEM, tiles * 2 * H, H};
        for (int k = 0; k < NQ; ++k) {
            most[k] = std::max(most[k], q[k]);
            if (bytes_per_sensor[s] > 0) per_byte[k] = std::max(per_byte[k], (double)q[k] / (double)bytes_per_sensor[s]);
        }
    }
    int64_t cap[NQ];
    for (int k = 0; k < NQ; ++k) {
        // plain launches run the frames one after another on one frame's workspace
        cap[k] = (plain ? 1 : (int64_t)max_frames) * most[k];
        if (budget > 0 && per_byte[k] > 0.0) cap[k] = std::min<int64_t>(cap[k], (int64_t)((double)budget * per_byte[k]) + most[k]);
    }
    CallTotals tot;
    tot.cells = cap[0];
    tot.tiles = cap[1];
    tot.vitems = cap[2];
    tot.border_slots = cap[3];
    tot.table_bytes = std::max(align_up(sizeof(BatchHeader) + sizeof(FrameDesc) * (size_t)max_frames, 8) + 8 * (size_t)cap[4],
                               (size_t)max_frames * align_up(sizeof(BatchHeader) + sizeof(FrameDesc) + 8 * (size_t)LIDAR_MAX_RINGS, 256));
    const hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return c->hip_fail(e, "hipSetDevice");
    return ensure_capacity(c, tot, stream);
}

extern "C" {

int lidar_mesh_segment(lidar_ctx* c, const lidar_frame_t* frames, int32_t n_frames,
                       const lidar_params_t* params, lidar_result_t* results, void* stream, int32_t launch) {
    return mesh_call(c, frames, n_frames, params, results, stream, launch, CALL_SEGMENT);
}

int lidar_mesh_normals(lidar_ctx* c, const lidar_frame_t* frames, int32_t n_frames,
                       const lidar_params_t* params, lidar_result_t* results, void* stream, int32_t launch) {
    return mesh_call(c, frames, n_frames, params, results, stream, launch, CALL_MESH_ONLY);
}

int lidar_label_grid(lidar_ctx* c, const lidar_frame_t* frames, int32_t n_frames,
                     const lidar_params_t* params, lidar_result_t* results, void* stream, int32_t launch) {
    return mesh_call(c, frames, n_frames, params, results, stream, launch, CALL_LABEL_GRID);
}

int lidar_mesh_segment_noalloc(lidar_ctx* c, const lidar_frame_t* frames, int32_t n_frames,
                               const lidar_params_t* params, lidar_result_t* results, void* stream,
                               int32_t launch) {
    return mesh_call_noalloc(c, frames, n_frames, params, results, stream, launch);
}

}  // extern "C"
