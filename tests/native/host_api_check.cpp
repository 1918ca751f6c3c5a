// host_api_check.cpp -- test driver for the C ABI with the host side built
// under AddressSanitizer (the kernels are built as usual).  Runs every entry
// point on small seeded synthetic sweeps on device 0: each launch form, the
// stage entry points, per-stage workgroup counts, the workspace limit, stage
// timing, argument errors and workspace growth; checks that the forms agree on
// the counts and outputs.  Exit status 0 = all checks passed; the sanitizer
// aborts on any invalid host access.  Built by tests/native/build.py.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lidarseg.h"

namespace {

int failures = 0;

void check(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

uint64_t rng = 0x9E3779B97F4A7C15ull;
double uniform() {  // xorshift64 in [0, 1)
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

// A sensor at the origin over the ground z = -1.7 and a wall y = 6.
std::vector<float> sweep(int H, int W, const std::vector<double>& elev, double drop) {
    std::vector<float> xyz;
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < W; ++j) {
        const double phi = 2.0 * pi * j / W;
        for (int i = 0; i < H; ++i) {
            if (uniform() < drop) continue;
            const double ux = std::cos(elev[i]) * std::cos(phi), uy = std::cos(elev[i]) * std::sin(phi),
                         uz = std::sin(elev[i]);
            double t = 1e30;
            if (uz < 0) t = std::fmin(t, -1.7 / uz);
            if (uy > 0) t = std::fmin(t, 6.0 / uy);
            if (t > 80.0) continue;
            t += 0.01 * (uniform() - 0.5);
            xyz.push_back((float)(t * ux));
            xyz.push_back((float)(t * uy));
            xyz.push_back((float)(t * uz));
        }
    }
    return xyz;
}

struct Frame {
    int H, W, s;
    std::vector<double> elev;
    lidar_sensor_t sensor;
    std::vector<float> host_xyz;
    float* xyz = nullptr;
    int64_t n = 0;
    int64_t maxV = 0, maxT = 0;
    // outputs
    float *vertices = nullptr, *normals = nullptr;
    int32_t *labels = nullptr, *triangles = nullptr, *vpoint = nullptr;
    int64_t* counts = nullptr;
};

void make_frame(Frame& f, int H, int W, int s, int wrap, double drop) {
    f.H = H;
    f.W = W;
    f.s = s;
    f.elev.resize(H);
    for (int i = 0; i < H; ++i) f.elev[i] = (H == 1 ? 0.0 : (10.0 - 30.0 * i / (H - 1))) * 3.14159265358979 / 180.0;
    f.sensor = lidar_sensor_t{H, W, s, wrap, f.elev.data(), 0.0};
    f.host_xyz = sweep(H, W, f.elev, drop);
    f.n = (int64_t)f.host_xyz.size() / 3;
    check(lidar_query_sizes(&f.sensor, &f.maxV, &f.maxT) == LIDAR_OK, "query sizes");
    (void)hipMalloc(&f.xyz, sizeof(float) * 3 * (f.n + 1));
    (void)hipMemcpy(f.xyz, f.host_xyz.data(), sizeof(float) * 3 * f.n, hipMemcpyHostToDevice);
    (void)hipMalloc(&f.vertices, sizeof(float) * 3 * f.maxV);
    (void)hipMalloc(&f.normals, sizeof(float) * 3 * f.maxV);
    (void)hipMalloc(&f.labels, sizeof(int32_t) * f.maxV);
    (void)hipMalloc(&f.triangles, sizeof(int32_t) * 3 * (f.maxT > 0 ? f.maxT : 1));
    (void)hipMalloc(&f.vpoint, sizeof(int32_t) * f.maxV);
    (void)hipMalloc(&f.counts, sizeof(int64_t) * 3);
}

void free_frame(Frame& f) {
    for (void* p : {(void*)f.xyz, (void*)f.vertices, (void*)f.normals, (void*)f.labels, (void*)f.triangles,
                    (void*)f.vpoint, (void*)f.counts})
        (void)hipFree(p);
}

struct Snapshot {
    int64_t counts[3];
    std::vector<float> normals;
    std::vector<int32_t> labels, triangles;
};

Snapshot snapshot(const Frame& f) {
    Snapshot s;
    (void)hipMemcpy(s.counts, f.counts, sizeof(s.counts), hipMemcpyDeviceToHost);
    const int64_t V = s.counts[0] > 0 ? s.counts[0] : 0, T = s.counts[1] > 0 ? s.counts[1] : 0;
    s.normals.resize(3 * V);
    s.labels.resize(V);
    s.triangles.resize(3 * T);
    if (V) {
        (void)hipMemcpy(s.normals.data(), f.normals, sizeof(float) * 3 * V, hipMemcpyDeviceToHost);
        (void)hipMemcpy(s.labels.data(), f.labels, sizeof(int32_t) * V, hipMemcpyDeviceToHost);
    }
    if (T) (void)hipMemcpy(s.triangles.data(), f.triangles, sizeof(int32_t) * 3 * T, hipMemcpyDeviceToHost);
    return s;
}

bool same(const Snapshot& a, const Snapshot& b, bool labels) {
    return std::memcmp(a.counts, b.counts, sizeof(int64_t) * (labels ? 3 : 2)) == 0 && a.normals == b.normals &&
           a.triangles == b.triangles && (!labels || a.labels == b.labels);
}

int run(lidar_ctx* ctx, std::vector<Frame>& fr, int launch, int (*call)(lidar_ctx*, const lidar_frame_t*, int32_t,
                                                                      const lidar_params_t*, lidar_result_t*, void*,
                                                                      int32_t),
        bool with_labels, const std::vector<float*>& normals_in = {}) {
    std::vector<lidar_frame_t> frames(fr.size());
    std::vector<lidar_result_t> results(fr.size());
    for (size_t k = 0; k < fr.size(); ++k) {
        frames[k] = lidar_frame_t{&fr[k].sensor, fr[k].xyz, fr[k].n,
                                  normals_in.empty() ? nullptr : normals_in[k], nullptr, nullptr};
        results[k] = lidar_result_t{fr[k].vertices, fr[k].normals, with_labels ? fr[k].labels : nullptr,
                                    fr[k].triangles, fr[k].vpoint, fr[k].counts, nullptr, nullptr};
    }
    lidar_params_t params{};
    params.r_min = 1.0;
    params.r_max = 60.0;
    params.thr[0] = params.thr[1] = params.thr[2] = 0.2;
    params.score_radius = 1;
    const int rc = call(ctx, frames.data(), (int32_t)fr.size(), &params, results.data(), nullptr, launch);
    (void)hipDeviceSynchronize();
    return rc;
}

}  // namespace

int main() {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        std::fprintf(stderr, "no HIP device\n");
        return 2;
    }
    lidar_ctx* ctx = nullptr;
    check(lidar_ctx_create(0, &ctx) == LIDAR_OK, "create");
    uint64_t held = 1;
    check(lidar_ctx_workspace_bytes(ctx, &held) == LIDAR_OK && held == 0, "empty workspace");

    std::vector<Frame> fr(4);
    make_frame(fr[0], 16, 360, 1, 1, 0.05);
    make_frame(fr[1], 33, 200, 2, 1, 0.2);
    make_frame(fr[2], 64, 256, 1, 0, 0.1);
    make_frame(fr[3], 5, 12, 1, 1, 0.0);

    // every launch form gives the same outputs
    check(run(ctx, fr, LIDAR_LAUNCH_PLAIN, lidar_mesh_segment, true) == LIDAR_OK, "plain");
    std::vector<Snapshot> ref;
    for (auto& f : fr) ref.push_back(snapshot(f));
    for (int launch : {LIDAR_LAUNCH_BATCHED, LIDAR_LAUNCH_GRAPH, LIDAR_LAUNCH_GRAPH}) {
        check(run(ctx, fr, launch, lidar_mesh_segment, true) == LIDAR_OK, "batched/graph");
        for (size_t k = 0; k < fr.size(); ++k) check(same(snapshot(fr[k]), ref[k], true), "forms agree");
    }
    // per-stage workgroups and tile shapes change nothing
    check(lidar_ctx_set_tuning(ctx, 300, 512, 256) == LIDAR_OK, "tuning");
    for (int st = 0; st < LIDAR_N_STAGES; ++st) check(lidar_ctx_set_stage_grid(ctx, st, 1 + 97 * st) == LIDAR_OK, "stage grid");
    for (int launch : {LIDAR_LAUNCH_BATCHED, LIDAR_LAUNCH_GRAPH}) {
        check(run(ctx, fr, launch, lidar_mesh_segment, true) == LIDAR_OK, "tuned run");
        for (size_t k = 0; k < fr.size(); ++k) check(same(snapshot(fr[k]), ref[k], true), "tuning agrees");
    }
    for (int st = 0; st < LIDAR_N_STAGES; ++st) (void)lidar_ctx_set_stage_grid(ctx, st, 0);
    (void)lidar_ctx_set_tuning(ctx, 0, 0, 0);
    // mesh and normals only: no labels written, same geometry
    for (int launch : {LIDAR_LAUNCH_PLAIN, LIDAR_LAUNCH_BATCHED, LIDAR_LAUNCH_GRAPH}) {
        check(run(ctx, fr, launch, lidar_mesh_normals, false) == LIDAR_OK, "mesh normals");
        for (size_t k = 0; k < fr.size(); ++k) {
            const Snapshot s = snapshot(fr[k]);
            check(same(s, ref[k], false) && s.counts[2] == 0, "mesh normals agree");
        }
    }
    // labels of given normals (the normals just computed)
    std::vector<float*> nin;
    for (auto& f : fr) {
        float* p = nullptr;
        (void)hipMalloc(&p, sizeof(float) * 3 * f.maxV);
        (void)hipMemcpy(p, f.normals, sizeof(float) * 3 * f.maxV, hipMemcpyDeviceToDevice);
        nin.push_back(p);
    }
    check(run(ctx, fr, LIDAR_LAUNCH_GRAPH, lidar_label_grid, true, nin) == LIDAR_OK, "label grid");
    for (size_t k = 0; k < fr.size(); ++k) check(same(snapshot(fr[k]), ref[k], true), "label grid agrees");
    check(run(ctx, fr, LIDAR_LAUNCH_GRAPH, lidar_label_grid, true) == LIDAR_EINVAL, "label grid needs normals");
    for (float* p : nin) (void)hipFree(p);

    // stage timing
    check(lidar_ctx_set_profiling(ctx, 1) == LIDAR_OK, "profiling on");
    check(run(ctx, fr, LIDAR_LAUNCH_BATCHED, lidar_mesh_segment, true) == LIDAR_OK, "profiled run");
    double ms[LIDAR_N_STAGES];
    int64_t n[LIDAR_N_STAGES];
    check(lidar_ctx_stage_times(ctx, ms, n) == LIDAR_OK && n[0] == 1 && ms[2] > 0.0, "stage times");
    (void)lidar_ctx_set_profiling(ctx, 0);

    // argument errors leave the context usable
    lidar_params_t bad{};
    bad.r_min = 5.0;
    bad.r_max = 1.0;
    lidar_frame_t f0{&fr[0].sensor, fr[0].xyz, fr[0].n, nullptr, nullptr, nullptr};
    lidar_result_t r0{fr[0].vertices, fr[0].normals, fr[0].labels, fr[0].triangles, nullptr, fr[0].counts,
                      nullptr, nullptr};
    check(lidar_mesh_segment(ctx, &f0, 1, &bad, &r0, nullptr, LIDAR_LAUNCH_BATCHED) == LIDAR_EINVAL, "bad range");
    check(std::strlen(lidar_ctx_last_error(ctx)) > 0, "error message");
    check(lidar_mesh_segment(ctx, &f0, 0, &bad, &r0, nullptr, LIDAR_LAUNCH_BATCHED) == LIDAR_EINVAL, "no frames");
    check(lidar_ctx_set_stage_grid(ctx, LIDAR_N_STAGES, 1) == LIDAR_EINVAL, "bad stage");
    check(lidar_ctx_set_tuning(ctx, 0, 768, 256) == LIDAR_EINVAL, "bad tile");

    // a workspace limit below what a larger batch needs refuses it; a fresh
    // context under the limit it needs runs it
    held = 0;
    check(lidar_ctx_workspace_bytes(ctx, &held) == LIDAR_OK && held > 0, "held");
    check(lidar_ctx_set_workspace_limit(ctx, held) == LIDAR_OK, "limit");
    std::vector<Frame> big(1);
    make_frame(big[0], 128, 2048, 1, 1, 0.1);
    check(run(ctx, big, LIDAR_LAUNCH_BATCHED, lidar_mesh_segment, true) == LIDAR_ENOMEM, "over the limit");
    check(lidar_ctx_set_workspace_limit(ctx, 0) == LIDAR_OK, "no limit");
    check(run(ctx, big, LIDAR_LAUNCH_BATCHED, lidar_mesh_segment, true) == LIDAR_OK, "growth");
    check(run(ctx, fr, LIDAR_LAUNCH_GRAPH, lidar_mesh_segment, true) == LIDAR_OK, "after growth");
    for (size_t k = 0; k < fr.size(); ++k) check(same(snapshot(fr[k]), ref[k], true), "after growth agrees");

    for (auto& f : fr) free_frame(f);
    free_frame(big[0]);
    lidar_ctx_destroy(ctx);
    std::printf("host api check: %d failures\n", failures);
    return failures ? 1 : 0;
}
