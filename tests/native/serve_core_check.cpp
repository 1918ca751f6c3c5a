// The served form's scheduler (paper_2005_02704_amd/csrc/serve_core.h) driven
// on the host by a fake executor with a hand-advanced clock: first come first
// served admission, group size, device-memory budget, buffer-set pools,
// completion, the watchdog, launch failures and releases.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "serve_core.h"

using lidarserve::Request;

namespace {

int g_failures = 0;

#define CHECK(cond)                                                         \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);     \
            ++g_failures;                                                   \
        }                                                                   \
    } while (0)

struct FakeExec {
    std::vector<std::vector<int32_t>> free_sets;  // per sensor
    std::vector<int> done;                        // per slot: 0 running, 1 finished, -1 failed
    std::vector<std::vector<int64_t>> launched;   // per slot: ids of its last group
    bool fail_next = false;
    int launches = 0;

    FakeExec(int n_sensors, int sets, int n_slots) : free_sets(n_sensors), done(n_slots, 0), launched(n_slots) {
        for (auto& p : free_sets)
            for (int k = 0; k < sets; ++k) p.push_back(k);
    }
    bool acquire_set(int32_t sensor, int32_t* set) {
        if (free_sets[sensor].empty()) return false;
        *set = free_sets[sensor].back();
        free_sets[sensor].pop_back();
        return true;
    }
    void return_set(int32_t sensor, int32_t set) { free_sets[sensor].push_back(set); }
    int launch(int slot, const Request* const* g, int n) {
        ++launches;
        launched[slot].clear();
        for (int i = 0; i < n; ++i) launched[slot].push_back(g[i]->id);
        done[slot] = 0;
        if (fail_next) {
            fail_next = false;
            return -1;
        }
        return 0;
    }
    int finished(int slot) { return done[slot]; }
};

Request req(int32_t sensor, uint64_t bytes) {
    Request r;
    r.sensor = sensor;
    r.bytes = bytes;
    r.n_points = 10;
    return r;
}

std::vector<Request> take(lidarserve::Scheduler<FakeExec>& s) {
    std::vector<Request> out(64);
    out.resize(s.take_done(out.data(), 64));
    return out;
}

void fifo_and_group_size() {
    FakeExec ex(1, 16, 2);
    lidarserve::Scheduler<FakeExec> s(ex, 2, 1000, 4, 0.0);
    for (int i = 0; i < 10; ++i) CHECK(s.submit(req(0, 1)) == i);
    CHECK(s.step(0.0) == 2);
    CHECK((ex.launched[0] == std::vector<int64_t>{0, 1, 2, 3}));
    CHECK((ex.launched[1] == std::vector<int64_t>{4, 5, 6, 7}));
    CHECK(s.step(0.1) == 0);  // both slots busy
    ex.done[0] = 1;
    CHECK(s.step(0.2) == 2);  // slot 0 completes, then takes 8 and 9
    CHECK((ex.launched[0] == std::vector<int64_t>{8, 9}));
    auto d = take(s);
    CHECK(d.size() == 4);
    for (size_t i = 0; i < d.size(); ++i) {
        CHECK(d[i].id == (int64_t)i);
        CHECK(d[i].status == lidarserve::ST_SERVED);
        CHECK(d[i].group_size == 4);
        CHECK(d[i].slot == 0);
        CHECK(d[i].t_done == 0.2);
    }
    Request r;
    CHECK(s.served(0, &r) && r.set >= 0);
    CHECK(s.release(0));
    CHECK(!s.release(0));  // released once
    CHECK(!s.release(5));  // still running
    ex.done[0] = ex.done[1] = 1;
    s.step(0.3);
    CHECK(take(s).size() == 6);
    CHECK(s.idle());
    for (int64_t id = 1; id < 10; ++id) CHECK(s.release(id));
    CHECK(ex.free_sets[0].size() == 16);
    auto st = s.stats();
    CHECK(st.groups == 3 && st.admitted == 10 && st.max_slots_busy == 2 && st.bytes_in_use == 0);
}

void budget() {
    FakeExec ex(1, 16, 3);
    lidarserve::Scheduler<FakeExec> s(ex, 3, 100, 8, 0.0);
    for (int i = 0; i < 5; ++i) s.submit(req(0, 40));
    s.step(0.0);
    // 80 bytes admitted into slot 0; the head (40 more) does not fit: nothing else is admitted
    CHECK(ex.launched[0].size() == 2 && ex.launched[1].empty() && ex.launched[2].empty());
    CHECK(s.stats().bytes_in_use == 80 && s.stats().peak_bytes == 80);
    ex.done[0] = 1;
    s.step(1.0);
    CHECK(ex.launched[0].size() == 2 && ex.launched[0][0] == 2);
    CHECK(s.stats().bytes_in_use == 80);
}

void buffer_sets() {
    // one set per sensor: a sensor's second request waits for the first's release,
    // and (first come first served) so do the requests behind it
    FakeExec ex(2, 1, 2);
    lidarserve::Scheduler<FakeExec> s(ex, 2, 1000, 8, 0.0);
    s.submit(req(0, 1));
    s.submit(req(0, 1));
    s.submit(req(1, 1));
    s.step(0.0);
    CHECK(ex.launched[0] == std::vector<int64_t>{0});
    CHECK(ex.launched[1].empty());
    ex.done[0] = 1;
    s.step(0.1);
    CHECK(take(s).size() == 1);
    s.step(0.2);
    CHECK(ex.launched[1].empty());  // request 1 still has no set
    CHECK(s.release(0));
    s.step(0.3);
    CHECK((ex.launched[0] == std::vector<int64_t>{1, 2}));
}

void watchdog() {
    FakeExec ex(1, 4, 1);
    lidarserve::Scheduler<FakeExec> s(ex, 1, 1000, 8, 1.0);
    s.submit(req(0, 1));
    s.submit(req(0, 1));
    s.step(0.0);
    s.step(0.5);
    CHECK(take(s).empty());
    s.submit(req(0, 1));
    s.step(1.5);  // overdue: its requests fail, the slot stays held
    auto d = take(s);
    CHECK(d.size() == 2);
    for (auto& r : d) CHECK(r.status == lidarserve::ST_TIMED_OUT && r.t_done == 1.5);
    CHECK(!s.release(0));  // timed out: nothing to release
    s.step(2.0);
    CHECK(take(s).empty());
    CHECK(ex.launches == 1);                 // request 2 waits for the slot
    CHECK(ex.free_sets[0].size() == 2);      // the timed-out group's sets are still held
    ex.done[0] = 1;                       // the device work ends
    s.step(2.5);
    CHECK(ex.launches == 2 && ex.launched[0] == std::vector<int64_t>{2});
    CHECK(ex.free_sets[0].size() == 3);      // two sets back, one taken by request 2
    CHECK(take(s).empty());                  // the late completion is not reported again
    CHECK(s.stats().timed_out == 2);
}

void timed_out_reports_outlive_their_records() {
    // the watchdog fires, then the device work ends (its sets return and the
    // records go) before anyone takes the reports: they must still be there
    FakeExec ex(1, 2, 1);
    lidarserve::Scheduler<FakeExec> s(ex, 1, 1000, 2, 1.0);
    s.submit(req(0, 1));
    s.submit(req(0, 1));
    s.step(0.0);
    s.step(2.0);               // overdue
    ex.done[0] = 1;
    s.step(2.5);               // the device finishes first
    auto d = take(s);
    CHECK(d.size() == 2);
    for (auto& r : d) CHECK(r.status == lidarserve::ST_TIMED_OUT && r.t_done == 2.0);
    CHECK(ex.free_sets[0].size() == 2);
    Request r;
    CHECK(!s.served(0, &r) && !s.release(0));
}

void device_failure() {
    // the device work of a group fails: its requests are reported failed, not
    // served, and their sets return at once
    FakeExec ex(1, 2, 1);
    lidarserve::Scheduler<FakeExec> s(ex, 1, 1000, 2, 0.0);
    s.submit(req(0, 1));
    s.submit(req(0, 1));
    s.step(0.0);
    ex.done[0] = -1;
    s.step(0.5);
    auto d = take(s);
    CHECK(d.size() == 2);
    for (auto& r : d) CHECK(r.status == lidarserve::ST_FAILED && r.t_done == 0.5);
    CHECK(ex.free_sets[0].size() == 2);
    CHECK(s.stats().failed == 2 && s.stats().bytes_in_use == 0);
    Request r;
    CHECK(!s.served(0, &r) && !s.release(0));
    CHECK(s.idle());
}

void launch_failure() {
    FakeExec ex(1, 4, 1);
    lidarserve::Scheduler<FakeExec> s(ex, 1, 1000, 8, 0.0);
    ex.fail_next = true;
    s.submit(req(0, 10));
    s.submit(req(0, 10));
    s.step(0.0);
    auto d = take(s);
    CHECK(d.size() == 2);
    for (auto& r : d) CHECK(r.status == lidarserve::ST_FAILED);
    CHECK(ex.free_sets[0].size() == 4);
    CHECK(s.stats().bytes_in_use == 0 && s.stats().failed == 2);
    CHECK(s.idle());
    s.submit(req(0, 10));
    s.step(0.1);
    CHECK(ex.launched[0] == std::vector<int64_t>{2});
}

}  // namespace

int main() {
    fifo_and_group_size();
    budget();
    buffer_sets();
    watchdog();
    timed_out_reports_outlive_their_records();
    device_failure();
    launch_failure();
    if (g_failures) {
        std::printf("%d checks failed\n", g_failures);
        return 1;
    }
    std::printf("serve_core: all checks passed\n");
    return 0;
}
