// Continuous-batching scheduler of the served form (plain C++, no HIP).
//
// Sweeps from several sensors arrive as requests.  Waiting requests are
// admitted first come first served into free slots -- a slot is one library
// context with its own stream -- as a group of at most max_batch requests, as
// long as the device memory the admitted groups hold stays within the budget
// and each request gets a free buffer set of its sensor.  A group runs as one
// batched call; requests that arrive while other groups are on the device join
// the next free slot, so groups overlap (continuous batching).  A watchdog
// fails a group's requests when the group runs longer than its limit, so no
// caller waits forever; the slot and the group's memory stay held until the
// device work really ends, since it may still write into them.
//
// The device side is a template parameter, so the scheduling logic runs on
// the host with a fake executor in the tests.  Exec provides
//   bool acquire_set(int32_t sensor, int32_t* set)  a free buffer set (false: none free now)
//   void return_set(int32_t sensor, int32_t set)
//   int  launch(int slot, const Request* const* group, int n)  enqueue; 0 on success
//   int  finished(int slot)   0 while the slot's group runs, 1 once it is done, -1 once its
//                             device work has failed (its requests fail)
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace lidarserve {

enum Status : int32_t {
    ST_WAITING = 0,    // queued
    ST_RUNNING = 1,    // admitted; its group is on the device
    ST_SERVED = 2,     // results are in its buffer set until released
    ST_TIMED_OUT = 3,  // the watchdog failed it; no results
    ST_FAILED = 4,     // its group could not be enqueued; no results
};

struct Request {
    int64_t id = -1;
    int32_t sensor = 0;
    const float* xyz = nullptr;  // host points of the sweep
    int64_t n_points = 0;
    uint64_t bytes = 0;          // device bytes the request holds while in flight
    double t_arrival = 0.0, t_admit = 0.0, t_done = 0.0;
    int32_t slot = -1, group = -1, group_size = 0;
    int32_t set = -1;            // buffer set (from admission until release)
    int32_t status = ST_WAITING;
};

template <class Exec>
class Scheduler {
public:
    Scheduler(Exec& ex, int n_slots, uint64_t budget, int max_batch, double timeout_s)
        : ex_(ex), slots_(n_slots), budget_(budget), max_batch_(max_batch), timeout_s_(timeout_s) {}

    // Queues a request; returns its id.  Thread-safe.
    int64_t submit(Request r) {
        std::lock_guard<std::mutex> lock(mu_);
        r.id = next_id_++;
        r.status = ST_WAITING;
        reqs_[r.id] = r;
        waiting_.push_back(r.id);
        return r.id;
    }

    // One pass of the loop at time `now`: finished groups complete, overdue
    // groups fail their requests, waiting requests are admitted into free
    // slots.  Returns the number of groups that changed state.
    int step(double now) {
        int changes = 0;
        for (int s = 0; s < (int)slots_.size(); ++s) {
            Slot& sl = slots_[s];
            if (!sl.busy) continue;
            const int fin = ex_.finished(s);
            if (fin != 0) {
                std::lock_guard<std::mutex> lock(mu_);
                for (int64_t id : sl.group) {
                    auto it = reqs_.find(id);
                    if (it == reqs_.end()) continue;
                    Request& r = it->second;
                    if (sl.abandoned) {
                        // reported as timed out already: its set returns now that the device is done
                        ex_.return_set(r.sensor, r.set);
                        reqs_.erase(it);
                    } else if (fin < 0) {
                        // the device work failed: no results, the set returns at once
                        ex_.return_set(r.sensor, r.set);
                        r.set = -1;
                        r.status = ST_FAILED;
                        r.t_done = now;
                        done_.push_back(r);
                        reqs_.erase(it);
                        ++failed_;
                    } else {
                        r.status = ST_SERVED;
                        r.t_done = now;
                        done_.push_back(r);
                    }
                }
                in_use_ -= sl.bytes;
                sl = Slot();
                ++changes;
            } else if (timeout_s_ > 0.0 && !sl.abandoned && now - sl.t_launch > timeout_s_) {
                std::lock_guard<std::mutex> lock(mu_);
                for (int64_t id : sl.group) {
                    Request& r = reqs_[id];
                    r.status = ST_TIMED_OUT;
                    r.t_done = now;
                    done_.push_back(r);
                    ++timed_out_;
                }
                sl.abandoned = true;
                ++changes;
            }
        }
        for (int s = 0; s < (int)slots_.size(); ++s) {
            if (slots_[s].busy) continue;
            std::vector<const Request*> group;
            uint64_t held = 0;
            {
                std::lock_guard<std::mutex> lock(mu_);
                while (!waiting_.empty() && (int)group.size() < max_batch_) {
                    Request& r = reqs_[waiting_.front()];
                    if (in_use_ + held + r.bytes > budget_) break;
                    int32_t set = -1;
                    if (!ex_.acquire_set(r.sensor, &set)) break;
                    waiting_.pop_front();
                    r.set = set;
                    r.status = ST_RUNNING;
                    r.t_admit = now;
                    r.slot = s;
                    r.group = groups_;
                    held += r.bytes;
                    group.push_back(&r);
                }
                if (group.empty()) break;  // first come first served: the head waits, so does the rest
                for (const Request* r : group) const_cast<Request*>(r)->group_size = (int32_t)group.size();
            }
            Slot& sl = slots_[s];
            sl.busy = true;
            sl.bytes = held;
            sl.t_launch = now;
            for (const Request* r : group) sl.group.push_back(r->id);
            // (the requests stay in the map until released: the pointers stay valid)
            const int rc = ex_.launch(s, group.data(), (int)group.size());
            std::lock_guard<std::mutex> lock(mu_);
            ++groups_;
            admitted_ += (int64_t)group.size();
            in_use_ += held;
            peak_in_use_ = std::max(peak_in_use_, in_use_);
            int busy = 0;
            for (const Slot& x : slots_) busy += x.busy ? 1 : 0;
            max_busy_ = std::max(max_busy_, busy);
            if (rc != 0) {
                for (int64_t id : sl.group) {
                    Request& r = reqs_[id];
                    ex_.return_set(r.sensor, r.set);
                    r.set = -1;
                    r.status = ST_FAILED;
                    r.t_done = now;
                    done_.push_back(r);
                    reqs_.erase(id);  // nothing held: forgotten at once
                    ++failed_;
                }
                in_use_ -= sl.bytes;
                sl = Slot();
            }
            ++changes;
        }
        return changes;
    }

    // Moves up to `max` finished requests (served, timed out or failed), as they
    // were when they finished, into `out`.  A report does not depend on the
    // request's record, which a timed-out request loses when its device work ends.
    int take_done(Request* out, int max) {
        std::lock_guard<std::mutex> lock(mu_);
        int n = 0;
        while (n < max && !done_.empty()) {
            out[n++] = done_.front();
            done_.pop_front();
        }
        return n;
    }

    // The request while it holds results (served, not yet released); nullptr otherwise.
    bool served(int64_t id, Request* out) {
        std::lock_guard<std::mutex> lock(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end() || it->second.status != ST_SERVED) return false;
        *out = it->second;
        return true;
    }

    // A served request's buffer set goes back to its pool.  False for an id
    // that is not served (unknown, waiting, running, timed out or failed).
    bool release(int64_t id) {
        std::lock_guard<std::mutex> lock(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end() || it->second.status != ST_SERVED) return false;
        ex_.return_set(it->second.sensor, it->second.set);
        reqs_.erase(it);
        return true;
    }

    // Nothing waiting and no group on the device.
    bool idle() {
        std::lock_guard<std::mutex> lock(mu_);
        if (!waiting_.empty()) return false;
        for (const Slot& s : slots_)
            if (s.busy) return false;
        return true;
    }
    bool anything_waiting() {
        std::lock_guard<std::mutex> lock(mu_);
        return !waiting_.empty();
    }

    struct Stats {
        int64_t groups, admitted, timed_out, failed;
        uint64_t peak_bytes, bytes_in_use;
        int32_t max_slots_busy;
    };
    Stats stats() {
        std::lock_guard<std::mutex> lock(mu_);
        return Stats{groups_, admitted_, timed_out_, failed_, peak_in_use_, in_use_, max_busy_};
    }

private:
    struct Slot {
        bool busy = false;
        bool abandoned = false;  // its requests failed on the watchdog; the device work still runs
        uint64_t bytes = 0;
        double t_launch = 0.0;
        std::vector<int64_t> group;
    };
    Exec& ex_;
    std::vector<Slot> slots_;
    const uint64_t budget_;
    const int max_batch_;
    const double timeout_s_;
    std::mutex mu_;
    std::unordered_map<int64_t, Request> reqs_;
    std::deque<int64_t> waiting_;
    std::deque<Request> done_;  // finished requests not yet taken, as they finished
    int64_t next_id_ = 0;
    uint64_t in_use_ = 0, peak_in_use_ = 0;
    int64_t groups_ = 0, admitted_ = 0, timed_out_ = 0, failed_ = 0;
    int32_t max_busy_ = 0;
};

}  // namespace lidarserve
