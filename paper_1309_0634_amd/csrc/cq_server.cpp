// Serving loop: many resident queries, batches that arrive over time.
//
// The paper's CPU side takes batches as they stream in, one iteration per
// batch, and keeps every group's window in GPU memory (Section 3.1,
// Section 3.2).  Here a server keeps many queries resident in HBM at once
// and takes their batches as requests:
//   - admission: a query is admitted only if its device footprint
//     (cq_query_footprint) fits the memory budget still free;
//   - lanes: a few HIP streams at the default priority.  Every query is
//     pinned to one lane, so its batches run in submission order; batches
//     of queries on different lanes overlap on the device;
//   - continuous batching: one launcher thread per lane starts the lane's
//     waiting requests in arrival order as soon as the lane has a free slot
//     (at most `slots` requests in flight per lane), while the caller keeps
//     submitting; lanes launch in parallel (the kernel launches happen
//     outside the lock) and sleep when they have nothing to start;
//   - completion: one reaper thread polls one event per request in flight
//     and records its latency (host clock from submission to the moment
//     its event is seen complete).
// A query object is only ever driven by its lane's launcher; the caller's
// threads touch the shared tables under one mutex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "cq.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    int64_t ticket;
    int32_t qid;
    const int32_t *keys, *values;
    int64_t n;
    int32_t *ids;
    int64_t *sums;
    int32_t *counts;
    double *avgs;
    int64_t *n_touched;
    Clock::time_point submitted;
    hipEvent_t done = nullptr;
    int lane = 0;
};

struct Entry {
    cq_query *q = nullptr;
    int lane = 0;
    int64_t bytes = 0;
    int64_t pending = 0;  // requests waiting or in flight
    bool removing = false;
};

struct Finished {
    int status;
    double latency_us;
};

}  // namespace

struct cq_server {
    int device = 0;
    int64_t budget = 0, used = 0;
    int32_t nlanes = 0, slots = 0;
    std::vector<hipStream_t> lanes;
    std::vector<int32_t> inflight_per_lane;
    std::map<int32_t, Entry> queries;
    int32_t next_qid = 0;
    int64_t next_ticket = 0;
    std::deque<Request> waiting;
    std::vector<Request> inflight;
    std::map<int64_t, Finished> finished;  // until waited for
    std::vector<hipEvent_t> spare_events;
    // statistics since the last cq_server_stats call
    std::vector<double> lat_us;
    int64_t stat_tuples = 0, stat_requests = 0;
    Clock::time_point stat_first{}, stat_last{};
    bool stat_open = false;
    std::mutex mu;
    std::condition_variable work;      // lane threads: a request or a free slot
    std::condition_variable launched;  // reaper: something is on the device
    std::condition_variable progress;  // callers: a request finished
    bool stop = false;
    std::vector<std::thread> dispatchers;  // one launcher per lane
    std::thread reaper;
};

namespace {

int from_hip(hipError_t e) {
    if (e == hipSuccess) return CQ_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return CQ_ERR_OOM;
    return CQ_ERR_HIP;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Starts request r on its lane.  Called by the lane's dispatcher with the
// lock held; releases it around the launches, so lanes launch in parallel
// and submissions are not held up.  The query cannot go away meanwhile
// (removal waits for its pending requests).
void launch(cq_server *s, std::unique_lock<std::mutex> &lk, Request r) {
    Entry &e = s->queries[r.qid];
    r.lane = e.lane;
    cq_query *q = e.q;
    hipStream_t st = s->lanes[e.lane];
    hipEvent_t ev = nullptr;
    if (!s->spare_events.empty()) {
        ev = s->spare_events.back();
        s->spare_events.pop_back();
    }
    s->inflight_per_lane[r.lane] += 1;
    s->inflight.push_back(r);  // listed (without an event yet) while it launches
    lk.unlock();
    int rc = CQ_OK;
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
        rc = CQ_ERR_HIP;
    }
    if (rc == CQ_OK)
        rc = cq_push_batch_results(q, r.keys, r.values, r.n, r.ids, r.sums, r.counts, r.avgs,
                                   r.n_touched, st);
    if (rc == CQ_OK && hipEventRecord(ev, st) != hipSuccess) rc = CQ_ERR_HIP;
    lk.lock();
    size_t i = 0;
    while (s->inflight[i].ticket != r.ticket) ++i;
    if (rc != CQ_OK) {  // finished at once, with the error
        if (ev) s->spare_events.push_back(ev);
        s->finished[r.ticket] = {rc, 0.0};
        s->inflight_per_lane[r.lane] -= 1;
        s->queries[r.qid].pending -= 1;
        s->inflight[i] = s->inflight.back();
        s->inflight.pop_back();
        s->progress.notify_all();
        return;
    }
    s->inflight[i].done = ev;
    s->launched.notify_one();
}

// Retires every in-flight request whose event has completed (lock held).
bool reap(cq_server *s) {
    bool any = false;
    for (size_t i = 0; i < s->inflight.size();) {
        Request &r = s->inflight[i];
        if (!r.done) {  // still launching
            ++i;
            continue;
        }
        const hipError_t q = hipEventQuery(r.done);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        const Clock::time_point now = Clock::now();
        const double us = std::chrono::duration<double, std::micro>(now - r.submitted).count();
        s->finished[r.ticket] = {q == hipSuccess ? CQ_OK : CQ_ERR_HIP, us};
        s->lat_us.push_back(us);
        s->stat_tuples += r.n;
        s->stat_requests += 1;
        if (!s->stat_open || r.submitted < s->stat_first) s->stat_first = r.submitted;
        if (!s->stat_open || now > s->stat_last) s->stat_last = now;
        s->stat_open = true;
        s->inflight_per_lane[r.lane] -= 1;
        s->queries[r.qid].pending -= 1;
        s->spare_events.push_back(r.done);
        s->inflight[i] = s->inflight.back();
        s->inflight.pop_back();
        any = true;
    }
    if (any) {
        s->progress.notify_all();
        s->work.notify_all();  // slots are free again
    }
    return any;
}

// Starts the oldest waiting request of `lane` if the lane has a free slot
// and no earlier request of the same query is still waiting (lock held;
// released around the launch).  Returns whether one was started.
bool admit_one(cq_server *s, std::unique_lock<std::mutex> &lk, int lane) {
    if (s->inflight_per_lane[lane] >= s->slots) return false;
    for (auto it = s->waiting.begin(); it != s->waiting.end(); ++it) {
        if (s->queries[it->qid].lane != lane) continue;
        // requests of one query sit on one lane in arrival order, so the
        // first one of this lane is never behind another of its query
        Request r = *it;
        s->waiting.erase(it);
        launch(s, lk, r);
        return true;
    }
    return false;
}

bool lane_idle(const cq_server *s, int lane) {
    if (s->inflight_per_lane[lane] > 0) return false;
    for (const Request &r : s->waiting)
        if (s->queries.at(r.qid).lane == lane) return false;
    return true;
}

// A lane's launcher: starts its lane's requests, sleeps when there is
// nothing to start.
void lane_loop(cq_server *s, int lane) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        if (admit_one(s, lk, lane)) continue;
        if (s->stop && lane_idle(s, lane)) break;
        s->work.wait(lk);
    }
}

// The reaper: polls the events of everything on the device (one thread
// spins, and only while something is in flight).
void reap_loop(cq_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        if (reap(s)) continue;
        if (s->stop && s->waiting.empty() && s->inflight.empty()) break;
        if (s->inflight.empty()) {
            s->launched.wait(lk);
        } else {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

}  // namespace

extern "C" {

int cq_server_create(int64_t memory_budget, int32_t lanes, int32_t slots, cq_server **out) {
    if (!out) return CQ_ERR_INVALID;
    *out = nullptr;
    if (memory_budget < 0 || lanes < 0 || lanes > CQ_SERVER_MAX_LANES || slots < 0 ||
        slots > CQ_SERVER_MAX_SLOTS)
        return CQ_ERR_INVALID;
    cq_server *s = new (std::nothrow) cq_server();
    if (!s) return CQ_ERR_OOM;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return CQ_ERR_HIP;
    }
    if (memory_budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return CQ_ERR_HIP;
        }
        memory_budget = (int64_t)(0.8 * (double)free_b);
    }
    s->budget = memory_budget;
    s->nlanes = lanes ? lanes : 8;
    s->slots = slots ? slots : 2;
    s->inflight_per_lane.assign(s->nlanes, 0);
    for (int i = 0; i < s->nlanes; ++i) {
        hipStream_t st = nullptr;
        // default priority, non-blocking with respect to the null stream
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->lanes) (void)hipStreamDestroy(x);
            delete s;
            return CQ_ERR_HIP;
        }
        s->lanes.push_back(st);
    }
    for (int i = 0; i < s->nlanes; ++i) s->dispatchers.emplace_back(lane_loop, s, i);
    s->reaper = std::thread(reap_loop, s);
    *out = s;
    return CQ_OK;
}

int cq_server_add_query(cq_server *s, int64_t groups, int32_t window, uint32_t aggregates,
                        int32_t *qid) {
    if (!s || !qid) return CQ_ERR_INVALID;
    const int64_t bytes = cq_query_footprint(groups, window);
    if (bytes < 0) return CQ_ERR_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->used + bytes > s->budget) return CQ_ERR_OOM;
        s->used += bytes;  // held while the query is created
    }
    DeviceGuard guard(s->device);
    cq_query *q = nullptr;
    const int rc = cq_create(groups, window, aggregates, &q);
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc != CQ_OK) {
        s->used -= bytes;
        return rc;
    }
    const int32_t id = s->next_qid++;
    Entry e;
    e.q = q;
    e.bytes = bytes;
    // the lane with the fewest queries
    std::vector<int> per(s->nlanes, 0);
    for (auto &kv : s->queries) per[kv.second.lane] += 1;
    e.lane = (int)(std::min_element(per.begin(), per.end()) - per.begin());
    s->queries[id] = e;
    *qid = id;
    return CQ_OK;
}

int cq_server_remove_query(cq_server *s, int32_t qid) {
    if (!s) return CQ_ERR_INVALID;
    cq_query *q = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->queries.find(qid);
        if (it == s->queries.end() || it->second.removing) return CQ_ERR_INVALID;
        it->second.removing = true;  // no new submissions
        s->progress.wait(lk, [&] { return s->queries[qid].pending == 0; });
        q = s->queries[qid].q;
        s->used -= s->queries[qid].bytes;
        s->queries.erase(qid);
    }
    DeviceGuard guard(s->device);
    return cq_destroy(q);
}

int cq_server_submit(cq_server *s, int32_t qid, const int32_t *keys, const int32_t *values,
                     int64_t n, int32_t *ids, int64_t *sums, int32_t *counts, double *avgs,
                     int64_t *n_touched, int64_t *ticket) {
    if (!s || !ticket || !n_touched || n < 0 || n > CQ_MAX_BATCH) return CQ_ERR_INVALID;
    if (n > 0 && (!keys || !values)) return CQ_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->queries.find(qid);
    if (it == s->queries.end() || it->second.removing || s->stop) return CQ_ERR_INVALID;
    Request r;
    r.ticket = s->next_ticket++;
    r.qid = qid;
    r.keys = keys;
    r.values = values;
    r.n = n;
    r.ids = ids;
    r.sums = sums;
    r.counts = counts;
    r.avgs = avgs;
    r.n_touched = n_touched;
    r.submitted = Clock::now();
    it->second.pending += 1;
    s->waiting.push_back(r);
    *ticket = r.ticket;
    s->work.notify_all();
    return CQ_OK;
}

int cq_server_wait(cq_server *s, int64_t ticket) {
    if (!s) return CQ_ERR_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket < 0) {  // everything submitted so far
        s->progress.wait(lk, [&] { return s->waiting.empty() && s->inflight.empty(); });
        int rc = CQ_OK;
        for (auto &kv : s->finished)
            if (kv.second.status != CQ_OK) rc = kv.second.status;
        s->finished.clear();
        return rc;
    }
    if (ticket >= s->next_ticket) return CQ_ERR_INVALID;
    bool known = s->finished.count(ticket) > 0;
    for (auto &r : s->waiting) known = known || r.ticket == ticket;
    for (auto &r : s->inflight) known = known || r.ticket == ticket;
    if (!known) return CQ_ERR_INVALID;  // waited for already
    s->progress.wait(lk, [&] { return s->finished.count(ticket) > 0; });
    const int rc = s->finished[ticket].status;
    s->finished.erase(ticket);
    return rc;
}

int cq_server_stats(cq_server *s, double *out) {
    if (!s || !out) return CQ_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> v = s->lat_us;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
        if (v.empty()) return 0.0;
        const size_t i = (size_t)std::min<double>((double)v.size() - 1, p * ((double)v.size() - 1) + 0.5);
        return v[i];
    };
    const double span =
        s->stat_open ? std::chrono::duration<double>(s->stat_last - s->stat_first).count() : 0.0;
    out[0] = (double)s->stat_requests;
    out[1] = pct(0.50);
    out[2] = pct(0.99);
    out[3] = v.empty() ? 0.0 : v.back();
    out[4] = (double)s->stat_tuples;
    out[5] = span > 0 ? (double)s->stat_tuples / span : 0.0;
    out[6] = (double)s->used;
    out[7] = (double)s->budget;
    s->lat_us.clear();
    s->stat_tuples = s->stat_requests = 0;
    s->stat_open = false;
    return CQ_OK;
}

int cq_server_destroy(cq_server *s) {
    if (!s) return CQ_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->work.notify_all();
        s->launched.notify_all();
    }
    for (std::thread &t : s->dispatchers)
        if (t.joinable()) t.join();  // each drains its lane first
    if (s->reaper.joinable()) s->reaper.join();
    DeviceGuard guard(s->device);
    int rc = CQ_OK;
    for (auto &kv : s->queries) {
        const int r = cq_destroy(kv.second.q);
        if (r != CQ_OK) rc = r;
    }
    for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
    for (hipStream_t st : s->lanes) (void)hipStreamDestroy(st);
    delete s;
    return rc;
}

}  // extern "C"
