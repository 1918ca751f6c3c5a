// Host side of the served form (include/lidarserve.h): the device executor of
// the scheduler in serve_core.h, the server thread and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lidarseg.h"
#include "lidarseg_internal.h"
#include "lidarserve.h"
#include "serve_core.h"

using lidarserve::Request;

namespace {

thread_local std::string g_serve_error;

struct SensorInfo {
    lidar_sensor_t s;
    std::vector<double> elev;
    int64_t V = 0, T = 0, rays = 0;
    uint64_t bytes = 0;  // device bytes one request of this sensor holds while in flight
};

// One resident buffer set of a sensor: device points and outputs, and the
// pinned host copies of the results.  Counts, labels and vertex points share
// one device block and one pinned block, so a sweep's results come back in one
// copy; in int32 words: [0, 6) counts (3 x int64), [8, 8 + Vc) labels,
// [8 + Vc, 8 + 2 Vc) vertex points.
struct BufferSet {
    float* d_xyz = nullptr;
    float* d_vertices = nullptr;
    float* d_normals = nullptr;
    int32_t* d_tris = nullptr;
    int32_t* d_block = nullptr;
    int32_t* h_block = nullptr;
    float* h_vertices = nullptr;  // copy_mesh only
    float* h_normals = nullptr;
    int32_t* h_tris = nullptr;
    int64_t Vc = 1, Tc = 1;
};

struct Executor {
    int device = 0;
    std::vector<lidar_ctx*> ctxs;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
    std::vector<SensorInfo> sensors;
    std::vector<std::vector<BufferSet>> sets;
    std::vector<std::vector<int32_t>> free_sets;  // guarded by the scheduler's lock
    std::vector<std::vector<lidar_frame_t>> frames;  // per slot, max_batch entries
    std::vector<std::vector<lidar_result_t>> results;
    lidar_params_t params{};
    int32_t launch_form = LIDAR_LAUNCH_GRAPH;
    bool copy_mesh = false;
    uint64_t device_bytes = 0;
    std::mutex err_mu;
    std::string err;  // the last launch failure

    bool acquire_set(int32_t sensor, int32_t* set) {
        auto& pool = free_sets[sensor];
        if (pool.empty()) return false;
        *set = pool.back();
        pool.pop_back();
        return true;
    }
    void return_set(int32_t sensor, int32_t set) { free_sets[sensor].push_back(set); }

    // One group on slot `slot`: the points in, lidar_mesh_segment over the
    // group, the results out, then the slot's event.
    int launch(int slot, const Request* const* g, int n) {
        hipStream_t st = streams[slot];
        lidar_frame_t* fr = frames[slot].data();
        lidar_result_t* rs = results[slot].data();
        for (int i = 0; i < n; ++i) {
            const Request& r = *g[i];
            BufferSet& b = sets[r.sensor][r.set];
            if (r.n_points > 0) {
                const hipError_t e = hipMemcpyAsync(b.d_xyz, r.xyz, 12 * (size_t)r.n_points, hipMemcpyHostToDevice, st);
                if (e != hipSuccess) return fail(std::string("points copy: ") + hipGetErrorString(e));
            }
            fr[i] = lidar_frame_t{&sensors[r.sensor].s, r.n_points > 0 ? b.d_xyz : nullptr, r.n_points,
                                  nullptr, nullptr, nullptr};
            rs[i] = lidar_result_t{b.d_vertices, b.d_normals, b.d_block + 8, b.d_tris, b.d_block + 8 + b.Vc,
                                   reinterpret_cast<int64_t*>(b.d_block), nullptr, nullptr};
        }
        const int rc = lidar_mesh_segment(ctxs[slot], fr, n, &params, rs, st, launch_form);
        if (rc != LIDAR_OK) return fail(std::string("lidar_mesh_segment: ") + lidar_ctx_last_error(ctxs[slot]));
        for (int i = 0; i < n; ++i) {
            const Request& r = *g[i];
            BufferSet& b = sets[r.sensor][r.set];
            hipError_t e = hipMemcpyAsync(b.h_block, b.d_block, sizeof(int32_t) * (8 + 2 * (size_t)b.Vc),
                                          hipMemcpyDeviceToHost, st);
            if (e == hipSuccess && copy_mesh) {
                e = hipMemcpyAsync(b.h_vertices, b.d_vertices, 12 * (size_t)b.Vc, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(b.h_normals, b.d_normals, 12 * (size_t)b.Vc, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(b.h_tris, b.d_tris, 12 * (size_t)b.Tc, hipMemcpyDeviceToHost, st);
            }
            if (e != hipSuccess) return fail(std::string("results copy: ") + hipGetErrorString(e));
        }
        const hipError_t e = hipEventRecord(done[slot], st);
        if (e != hipSuccess) return fail(std::string("hipEventRecord: ") + hipGetErrorString(e));
        return 0;
    }

    // 0 while the slot's group runs, 1 once it is done, -1 if its device work failed.
    int finished(int slot) {
        const hipError_t e = hipEventQuery(done[slot]);
        if (e == hipErrorNotReady) return 0;
        if (e == hipSuccess) return 1;
        fail(std::string("group on slot ") + std::to_string(slot) + ": " + hipGetErrorString(e));
        return -1;
    }

    int fail(const std::string& msg) {
        std::lock_guard<std::mutex> lock(err_mu);
        err = msg;
        return -1;
    }
};

}  // namespace

struct lidar_server {
    int device = 0;
    Executor ex;
    std::unique_ptr<lidarserve::Scheduler<Executor>> sched;
    std::thread thread;
    std::atomic<bool> stop{false};
    std::atomic<bool> pending{false};
    std::mutex cv_mu;
    std::condition_variable cv;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    uint64_t budget = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    // Failures are reported per calling thread (any thread may call the server).
    int fail(int code, const std::string& msg) {
        g_serve_error = msg;
        return code;
    }
};

namespace {

// The server thread: scheduling passes while groups run or requests wait; a
// wait on the condition variable (woken by submissions) when idle.
void serve_loop(lidar_server* s) {
    (void)hipSetDevice(s->device);
    while (!s->stop.load(std::memory_order_acquire)) {
        if (s->sched->step(s->now())) continue;
        if (s->sched->idle()) {
            std::unique_lock<std::mutex> lock(s->cv_mu);
            s->cv.wait_for(lock, std::chrono::milliseconds(1),
                           [&] { return s->stop.load() || s->pending.load(); });
            s->pending.store(false);
        } else {
            std::this_thread::yield();
        }
    }
}

void free_server(lidar_server* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    for (auto st : s->ex.streams)
        if (st) (void)hipStreamSynchronize(st);
    for (auto c : s->ex.ctxs)
        if (c) lidar_ctx_destroy(c);
    for (auto& pool : s->ex.sets)
        for (auto& b : pool) {
            for (void* p : {(void*)b.d_xyz, (void*)b.d_vertices, (void*)b.d_normals, (void*)b.d_tris, (void*)b.d_block})
                if (p) (void)hipFree(p);
            for (void* p : {(void*)b.h_block, (void*)b.h_vertices, (void*)b.h_normals, (void*)b.h_tris})
                if (p) (void)hipHostFree(p);
        }
    for (auto ev : s->ex.done)
        if (ev) (void)hipEventDestroy(ev);
    for (auto st : s->ex.streams)
        if (st) (void)hipStreamDestroy(st);
    delete s;
}

}  // namespace

extern "C" {

const char* lidar_server_last_error(const lidar_server*) { return g_serve_error.c_str(); }

double lidar_server_now(const lidar_server* srv) { return srv ? srv->now() : 0.0; }

int lidar_server_create(int device, const lidar_sensor_t* sensors, int32_t n_sensors, const lidar_params_t* params,
                        const lidar_server_opts_t* opts, lidar_server** out) {
    if (!out) { g_serve_error = "out is NULL"; return LIDAR_EINVAL; }
    *out = nullptr;
    if (!sensors || n_sensors < 1 || !params || !opts) { g_serve_error = "need sensors, params and opts"; return LIDAR_EINVAL; }
    const lidar_server_opts_t& o = *opts;
    if (o.n_slots < 1 || o.n_slots > 16) { g_serve_error = "n_slots must lie in [1, 16]"; return LIDAR_EINVAL; }
    if (o.max_batch < 1 || o.max_batch > 256) { g_serve_error = "max_batch must lie in [1, 256]"; return LIDAR_EINVAL; }
    if (o.launch != LIDAR_LAUNCH_PLAIN && o.launch != LIDAR_LAUNCH_BATCHED && o.launch != LIDAR_LAUNCH_GRAPH) {
        g_serve_error = "unknown launch form";
        return LIDAR_EINVAL;
    }
    if (o.sets_per_sensor < 1) { g_serve_error = "sets_per_sensor must be >= 1"; return LIDAR_EINVAL; }
    if (o.budget_bytes == 0) { g_serve_error = "budget_bytes must be > 0"; return LIDAR_EINVAL; }
    if (!(o.timeout_s >= 0.0)) { g_serve_error = "timeout_s must be >= 0"; return LIDAR_EINVAL; }
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) { g_serve_error = hipGetErrorString(e); return LIDAR_EINVAL; }

    lidar_server* s = new lidar_server();
    s->device = device;
    s->budget = o.budget_bytes;
    Executor& ex = s->ex;
    ex.device = device;
    ex.params = *params;
    ex.launch_form = o.launch;
    ex.copy_mesh = o.copy_mesh != 0;
    ex.sensors.resize(n_sensors);
    for (int q = 0; q < n_sensors; ++q) {
        SensorInfo& si = ex.sensors[q];
        si.s = sensors[q];
        int64_t V = 0, T = 0;
        const int rc = lidar_query_sizes(&sensors[q], &V, &T);
        if (rc) {
            const std::string msg = "sensor " + std::to_string(q) + ": " + lidar_last_error();
            free_server(s);
            g_serve_error = msg;
            return rc;
        }
        si.elev.assign(sensors[q].elev_rad, sensors[q].elev_rad + sensors[q].n_rings);
        si.s.elev_rad = si.elev.data();
        si.V = V;
        si.T = T;
        si.rays = (int64_t)sensors[q].n_rings * sensors[q].n_azimuth;
        // points, outputs (vertices, normals, labels, vertex points, triangles),
        // key grid and other workspace of the sweep
        si.bytes = 12 * (uint64_t)si.rays + 36 * (uint64_t)V + 12 * (uint64_t)T + 8 * (uint64_t)V + 16 * (uint64_t)V;
    }
    // contexts, streams, events
    for (int k = 0; k < o.n_slots; ++k) {
        lidar_ctx* c = nullptr;
        int rc = lidar_ctx_create(device, &c);
        if (rc) { free_server(s); g_serve_error = std::string("context: ") + lidar_last_error(); return rc; }
        ex.ctxs.push_back(c);
        if (o.tile_cells || o.tile_threads || o.grid) {
            rc = lidar_ctx_set_tuning(c, o.grid, o.tile_cells, o.tile_threads);
            if (rc) { const std::string m = lidar_ctx_last_error(c); free_server(s); g_serve_error = m; return rc; }
        }
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            if (st) (void)hipStreamDestroy(st);
            free_server(s);
            g_serve_error = "cannot create streams and events";
            return LIDAR_EDEVICE;
        }
        ex.streams.push_back(st);
        ex.done.push_back(ev);
        ex.frames.emplace_back(o.max_batch);
        ex.results.emplace_back(o.max_batch);
    }
    // each slot's workspace, for the largest group the budget admits
    {
        std::vector<lidar_sensor_t> ss(n_sensors);
        std::vector<uint64_t> bytes(n_sensors);
        for (int q = 0; q < n_sensors; ++q) {
            ss[q] = ex.sensors[q].s;
            bytes[q] = ex.sensors[q].bytes;
        }
        for (int k = 0; k < o.n_slots; ++k) {
            const int rc = lidarseg::ctx_reserve(ex.ctxs[k], ss.data(), n_sensors, o.max_batch, o.budget_bytes,
                                                 bytes.data(), o.launch == LIDAR_LAUNCH_PLAIN, ex.streams[k]);
            if (rc) {
                const std::string m = std::string("workspace: ") + lidar_ctx_last_error(ex.ctxs[k]);
                free_server(s);
                g_serve_error = m;
                return rc;
            }
        }
    }
    // buffer sets
    ex.sets.resize(n_sensors);
    ex.free_sets.resize(n_sensors);
    for (int q = 0; q < n_sensors; ++q) {
        const SensorInfo& si = ex.sensors[q];
        for (int k = 0; k < o.sets_per_sensor; ++k) {
            BufferSet b;
            b.Vc = std::max<int64_t>(si.V, 1);
            b.Tc = std::max<int64_t>(si.T, 1);
            bool ok = hipMalloc(&b.d_xyz, 12 * (size_t)std::max<int64_t>(si.rays, 1)) == hipSuccess &&
                      hipMalloc(&b.d_vertices, 12 * (size_t)b.Vc) == hipSuccess &&
                      hipMalloc(&b.d_normals, 12 * (size_t)b.Vc) == hipSuccess &&
                      hipMalloc(&b.d_tris, 12 * (size_t)b.Tc) == hipSuccess &&
                      hipMalloc(&b.d_block, sizeof(int32_t) * (8 + 2 * (size_t)b.Vc)) == hipSuccess &&
                      hipHostMalloc(&b.h_block, sizeof(int32_t) * (8 + 2 * (size_t)b.Vc), hipHostMallocDefault) == hipSuccess;
            if (ok && ex.copy_mesh)
                ok = hipHostMalloc(&b.h_vertices, 12 * (size_t)b.Vc, hipHostMallocDefault) == hipSuccess &&
                     hipHostMalloc(&b.h_normals, 12 * (size_t)b.Vc, hipHostMallocDefault) == hipSuccess &&
                     hipHostMalloc(&b.h_tris, 12 * (size_t)b.Tc, hipHostMallocDefault) == hipSuccess;
            ex.sets[q].push_back(b);
            if (!ok) { free_server(s); g_serve_error = "cannot allocate the buffer sets"; return LIDAR_ENOMEM; }
            ex.device_bytes += 12 * (uint64_t)std::max<int64_t>(si.rays, 1) + 24 * (uint64_t)b.Vc + 12 * (uint64_t)b.Tc +
                               4 * (8 + 2 * (uint64_t)b.Vc);
            ex.free_sets[q].push_back(k);
        }
    }
    for (auto c : ex.ctxs) {
        uint64_t held = 0;
        if (lidar_ctx_workspace_bytes(c, &held) == LIDAR_OK) ex.device_bytes += held;
    }
    // one empty group per slot: the graph is captured (and every lazily made
    // object exists) before serving starts
    for (int k = 0; k < o.n_slots; ++k) {
        Request r;
        r.sensor = 0;
        r.n_points = 0;
        r.set = 0;
        const Request* g[1] = {&r};
        if (ex.launch(k, g, 1) != 0 || hipStreamSynchronize(ex.streams[k]) != hipSuccess) {
            const std::string m = "warm-up group: " + ex.err;
            free_server(s);
            g_serve_error = m;
            return LIDAR_EDEVICE;
        }
    }
    s->sched.reset(new lidarserve::Scheduler<Executor>(ex, o.n_slots, o.budget_bytes, o.max_batch, o.timeout_s));
    s->thread = std::thread(serve_loop, s);
    *out = s;
    return LIDAR_OK;
}

void lidar_server_destroy(lidar_server* s) {
    if (!s) return;
    s->stop.store(true, std::memory_order_release);
    s->cv.notify_all();
    if (s->thread.joinable()) s->thread.join();
    free_server(s);
}

int lidar_server_submit(lidar_server* s, int32_t sensor, const float* xyz, int64_t n_points, int64_t* id) {
    if (!s || !id) { g_serve_error = "server or id is NULL"; return LIDAR_EINVAL; }
    if (sensor < 0 || sensor >= (int32_t)s->ex.sensors.size()) return s->fail(LIDAR_EINVAL, "no such sensor");
    const SensorInfo& si = s->ex.sensors[sensor];
    if (n_points < 0 || n_points > si.rays)
        return s->fail(LIDAR_EINVAL, "n_points must lie in [0, n_rings * n_azimuth] of the sensor");
    if (n_points > 0 && !xyz) return s->fail(LIDAR_EINVAL, "xyz is NULL");
    if (si.bytes > s->budget) return s->fail(LIDAR_EINVAL, "one sweep of this sensor needs more than the budget");
    Request r;
    r.sensor = sensor;
    r.xyz = xyz;
    r.n_points = n_points;
    r.bytes = si.bytes;
    r.t_arrival = s->now();
    *id = s->sched->submit(r);
    s->pending.store(true);
    s->cv.notify_one();
    return LIDAR_OK;
}

int lidar_server_poll(lidar_server* s, lidar_served_t* done, int32_t max, int32_t* n_done) {
    if (!s || !n_done || (max > 0 && !done)) { g_serve_error = "bad arguments"; return LIDAR_EINVAL; }
    *n_done = 0;
    if (max <= 0) return LIDAR_OK;
    std::vector<Request> got(std::min<int32_t>(max, 4096));
    const int n = s->sched->take_done(got.data(), (int)got.size());
    for (int i = 0; i < n; ++i) {
        const Request& r = got[i];
        done[i] = lidar_served_t{r.id, r.sensor, r.status, r.slot, r.group_size, r.t_arrival, r.t_admit, r.t_done};
    }
    *n_done = n;
    return LIDAR_OK;
}

int lidar_server_result(lidar_server* s, int64_t id, lidar_server_result_t* out) {
    if (!s || !out) { g_serve_error = "server or out is NULL"; return LIDAR_EINVAL; }
    Request r;
    if (!s->sched->served(id, &r)) return s->fail(LIDAR_EINVAL, "request " + std::to_string(id) + " holds no results");
    const BufferSet& b = s->ex.sets[r.sensor][r.set];
    out->counts = reinterpret_cast<const int64_t*>(b.h_block);
    out->labels = b.h_block + 8;
    out->vertex_point = b.h_block + 8 + b.Vc;
    out->vertices = b.h_vertices;
    out->normals = b.h_normals;
    out->triangles = b.h_tris;
    return LIDAR_OK;
}

int lidar_server_release(lidar_server* s, int64_t id) {
    if (!s) { g_serve_error = "server is NULL"; return LIDAR_EINVAL; }
    if (!s->sched->release(id)) return s->fail(LIDAR_EINVAL, "request " + std::to_string(id) + " holds no results");
    s->pending.store(true);  // a set came free: a waiting request may now be admitted
    s->cv.notify_one();
    return LIDAR_OK;
}

int lidar_server_stats(lidar_server* s, lidar_server_stats_t* out) {
    if (!s || !out) { g_serve_error = "server or out is NULL"; return LIDAR_EINVAL; }
    const auto st = s->sched->stats();
    *out = lidar_server_stats_t{st.groups, st.admitted, st.timed_out, st.failed, st.peak_bytes, st.max_slots_busy,
                                s->ex.device_bytes};
    return LIDAR_OK;
}

int lidar_server_replay(lidar_server* s, int64_t n, const double* t_offset, const int32_t* sensor,
                        const float* const* xyz, const int64_t* n_points, double* latency_s, int32_t* status,
                        int32_t* group_size, double* wall_s) {
    if (!s || n < 0 || (n > 0 && (!t_offset || !sensor || !xyz || !n_points))) {
        g_serve_error = "bad arguments";
        return LIDAR_EINVAL;
    }
    std::vector<int64_t> ids(n, -1);
    std::unordered_map<int64_t, int64_t> index;  // request id -> position in the schedule
    index.reserve((size_t)n * 2);
    std::vector<lidar_served_t> done(256);
    int64_t finished = 0, next = 0;
    const double start = s->now();
    auto drain = [&]() {
        int32_t k = 0;
        (void)lidar_server_poll(s, done.data(), (int32_t)done.size(), &k);
        for (int32_t j = 0; j < k; ++j) {
            const lidar_served_t& d = done[j];
            auto it = index.find(d.id);
            if (it == index.end()) continue;  // not one of ours
            const int64_t i = it->second;
            if (latency_s) latency_s[i] = d.t_done - d.t_arrival;
            if (status) status[i] = d.status;
            if (group_size) group_size[i] = d.group_size;
            if (d.status == LIDAR_SERVED_OK) (void)lidar_server_release(s, d.id);
            ++finished;
        }
        return k;
    };
    while (finished < n) {
        // submit every request whose time has come
        while (next < n && s->now() - start >= t_offset[next]) {
            int64_t id = -1;
            const int rc = lidar_server_submit(s, sensor[next], xyz[next], n_points[next], &id);
            if (rc) return rc;
            ids[next] = id;
            index[id] = next;
            ++next;
        }
        if (drain() == 0) {
            const double wait = next < n ? t_offset[next] - (s->now() - start) : 0.0;
            if (wait > 2e-4)
                std::this_thread::sleep_for(std::chrono::microseconds((int64_t)((wait - 1e-4) * 1e6)));
            else
                std::this_thread::yield();
        }
    }
    if (wall_s) *wall_s = s->now() - start;
    return LIDAR_OK;
}

}  // extern "C"
