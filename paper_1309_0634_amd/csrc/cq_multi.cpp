// Many queries over one input stream, with an online autotuner.
//
// Every batch is handed to all queries of the set (each typically reducing
// keys mod its own group count, cq_set_key_mod).  The queries are spread
// over a few HIP streams ("lanes", default priority) forked from and joined
// back into the caller's stream with events, so queries on different lanes
// overlap on the device while each query's own batches stay in order.
//
// The autotuner works on live batches: every partition gives identical
// results (the balancer moves no state), so candidates can be tried on the
// real stream with nothing to undo.  During the tuning window each query
// runs each of its candidates -- the balanced partition and the static
// partition with 1024 and with 4096 workers where they are allowed -- for
// `reps` batches, timed with events around its launches on its lane.  Then
// every query keeps its fastest candidate (median time), and the queries
// are re-spread over the lanes longest first, each to the lane with the
// least time so far (LPT scheduling), so that the lanes finish together.
// The paper's lesson that the partition granularity decides how much skew
// hurts (Section 5.2, the grid-size experiment) is what the candidates
// cover.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <numeric>
#include <vector>

#include "cq.h"
#include "cq_internal.h"

namespace {

struct Cand {
    int32_t mode, workers;
};

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

}  // namespace

struct cq_multi {
    int device = 0;
    std::vector<cq_query *> qs;
    std::vector<int64_t> groups;
    std::vector<hipStream_t> lanes;
    std::vector<int> lane_of;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    // tuning
    int32_t reps = 0;
    int32_t tune_step = 0, tune_len = 0;  // pushes done / in the window
    std::vector<std::vector<Cand>> cands;
    std::vector<std::vector<std::vector<float>>> times;  // [query][candidate] ms
    std::vector<hipEvent_t> t0, t1;                     // per query
    std::vector<int> chosen;
    std::vector<float> chosen_ms;
    // graph replay: the set's whole per-batch launch sequence, captured
    // once per batch size, reads the batch from staging buffers
    bool graph = false;
    hipStream_t origin = nullptr;
    int32_t *keys_st = nullptr, *vals_st = nullptr;
    int64_t st_cap = 0;
    std::vector<std::pair<int64_t, hipGraphExec_t>> execs;
};

namespace {

bool static_allowed(int64_t G, int32_t w) { return (G + w - 1) / w <= 2048; }

int from_hip(hipError_t e) { return e == hipSuccess ? CQ_OK : CQ_ERR_HIP; }

// The candidate query i runs at tuning push `step`.
int cand_at(const cq_multi *m, int i, int step) {
    return (step / m->reps) % (int)m->cands[i].size();
}

void drop_graphs(cq_multi *m) {
    for (auto &e : m->execs) (void)hipGraphExecDestroy(e.second);
    m->execs.clear();
}

// Enqueues one batch on every query, lane by lane (eager, or while the
// origin stream is being captured).
int enqueue_all(cq_multi *m, const int32_t *keys, const int32_t *values, int64_t n,
                hipStream_t s, bool tuning) {
    const int nq = (int)m->qs.size();
    hipError_t e = hipEventRecord(m->fork, s);
    for (hipStream_t l : m->lanes)
        if (e == hipSuccess) e = hipStreamWaitEvent(l, m->fork, 0);
    int rc = from_hip(e);
    // lane by lane, so each lane's launches are issued back to back
    for (int l = 0; l < (int)m->lanes.size() && rc == CQ_OK; ++l) {
        for (int i = 0; i < nq && rc == CQ_OK; ++i) {
            if (m->lane_of[i] != l) continue;
            if (tuning) {
                const Cand c = m->cands[i][cand_at(m, i, m->tune_step)];
                rc = cq_set_partition(m->qs[i], c.mode, c.workers);
                if (rc == CQ_OK) rc = from_hip(hipEventRecord(m->t0[i], m->lanes[l]));
            }
            if (rc == CQ_OK) rc = cq_push_batch(m->qs[i], keys, values, n, m->lanes[l]);
            if (rc == CQ_OK && tuning) rc = from_hip(hipEventRecord(m->t1[i], m->lanes[l]));
        }
        if (rc == CQ_OK) rc = from_hip(hipEventRecord(m->joins[l], m->lanes[l]));
        if (rc == CQ_OK) rc = from_hip(hipStreamWaitEvent(s, m->joins[l], 0));
    }
    return rc;
}

// Graph push: copy the batch to staging, then replay the captured sequence
// for this size (capturing it the first time).
int graph_push(cq_multi *m, const int32_t *keys, const int32_t *values, int64_t n,
               hipStream_t s) {
    if (n > m->st_cap) {  // larger staging: every captured graph read the old one
        drop_graphs(m);
        if (hipStreamSynchronize(s) != hipSuccess) return CQ_ERR_HIP;
        if (m->keys_st) (void)hipFree(m->keys_st);
        if (m->vals_st) (void)hipFree(m->vals_st);
        m->keys_st = m->vals_st = nullptr;
        m->st_cap = 0;
        if (hipMalloc(&m->keys_st, sizeof(int32_t) * (size_t)n) != hipSuccess ||
            hipMalloc(&m->vals_st, sizeof(int32_t) * (size_t)n) != hipSuccess)
            return CQ_ERR_OOM;
        m->st_cap = n;
    }
    const size_t bytes = sizeof(int32_t) * (size_t)n;
    if (n > 0 &&
        (hipMemcpyAsync(m->keys_st, keys, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
         hipMemcpyAsync(m->vals_st, values, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess))
        return CQ_ERR_HIP;
    for (auto &e : m->execs)
        if (e.first == n) {
            for (cq_query *q : m->qs) cq::query_replayed(q, n, s);
            return from_hip(hipGraphLaunch(e.second, s));
        }
    // capture: the pushes run their host logic now (each query's sequence
    // number moves on), their launches go into the graph, and the launch
    // below performs them
    for (cq_query *q : m->qs) {
        const int rc = cq::query_set_graph(q, true, s);
        if (rc != CQ_OK) return rc;
    }
    hipEvent_t ready = nullptr;
    if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return CQ_ERR_HIP;
    hipError_t e = hipEventRecord(ready, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(m->origin, ready, 0);
    if (e == hipSuccess) e = hipStreamBeginCapture(m->origin, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipEventDestroy(ready);
        return CQ_ERR_HIP;
    }
    const int rc = enqueue_all(m, m->keys_st, m->vals_st, n, m->origin, false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(m->origin, &g);
    (void)hipEventDestroy(ready);
    if (rc != CQ_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != CQ_OK ? rc : CQ_ERR_HIP;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return CQ_ERR_HIP;
    m->execs.push_back({n, x});
    for (cq_query *q : m->qs) cq::query_ran_on(q, s);  // the work runs on s, not on a lane
    return from_hip(hipGraphLaunch(x, s));
}

// After the tuning window: fastest candidate per query, lanes by LPT.
void finish_tuning(cq_multi *m) {
    const int nq = (int)m->qs.size();
    m->chosen.assign(nq, 0);
    m->chosen_ms.assign(nq, 0.f);
    for (int i = 0; i < nq; ++i) {
        float best = 0.f;
        int bi = 0;
        for (int c = 0; c < (int)m->cands[i].size(); ++c) {
            std::vector<float> v = m->times[i][c];
            if (v.empty()) continue;
            std::sort(v.begin(), v.end());
            const float med = v[v.size() / 2];
            if (c == 0 || med < best) {
                best = med;
                bi = c;
            }
        }
        m->chosen[i] = bi;
        m->chosen_ms[i] = best;
        (void)cq_set_partition(m->qs[i], m->cands[i][bi].mode, m->cands[i][bi].workers);
    }
    std::vector<int> order(nq);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return m->chosen_ms[a] > m->chosen_ms[b]; });
    std::vector<double> load(m->lanes.size(), 0.0);
    for (int i : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        m->lane_of[i] = l;
        load[l] += m->chosen_ms[i];
    }
}

}  // namespace

extern "C" {

int cq_multi_create(cq_query *const *queries, int32_t count, int32_t lanes, cq_multi **out) {
    if (!out) return CQ_ERR_INVALID;
    *out = nullptr;
    if (!queries || count < 1 || lanes < 0 || lanes > CQ_MULTI_MAX_LANES) return CQ_ERR_INVALID;
    for (int i = 0; i < count; ++i)
        if (!queries[i]) return CQ_ERR_INVALID;
    cq_multi *m = new (std::nothrow) cq_multi();
    if (!m) return CQ_ERR_OOM;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return CQ_ERR_HIP;
    }
    const int nl = std::min<int>(lanes ? lanes : 8, count);
    hipError_t e = hipEventCreateWithFlags(&m->fork, hipEventDisableTiming);
    for (int l = 0; l < nl && e == hipSuccess; ++l) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) break;
        m->lanes.push_back(s);
        hipEvent_t j = nullptr;
        e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        if (e == hipSuccess) m->joins.push_back(j);
    }
    for (int i = 0; i < count && e == hipSuccess; ++i) {
        m->qs.push_back(queries[i]);
        int64_t G = 0;
        e = cq_query_groups(queries[i], &G) == CQ_OK ? hipSuccess : hipErrorInvalidValue;
        m->groups.push_back(G);
        m->lane_of.push_back(i % nl);
    }
    if (e != hipSuccess) {
        (void)cq_multi_destroy(m);
        return from_hip(e);
    }
    *out = m;
    return CQ_OK;
}

int cq_multi_tune(cq_multi *m, int32_t reps) {
    if (!m || reps < 1 || reps > 64) return CQ_ERR_INVALID;
    DeviceGuard guard(m->device);
    const int nq = (int)m->qs.size();
    m->reps = reps;
    m->cands.assign(nq, {});
    int most = 1;
    for (int i = 0; i < nq; ++i) {
        m->cands[i].push_back({CQ_PARTITION_BALANCED, 0});
        for (int32_t w : {1024, 4096})
            if (static_allowed(m->groups[i], w)) m->cands[i].push_back({CQ_PARTITION_STATIC, w});
        most = std::max<int>(most, (int)m->cands[i].size());
    }
    m->times.assign(nq, {});
    for (int i = 0; i < nq; ++i) m->times[i].assign(m->cands[i].size(), {});
    if (m->t0.empty()) {
        m->t0.resize(nq);
        m->t1.resize(nq);
        for (int i = 0; i < nq; ++i)
            if (hipEventCreate(&m->t0[i]) != hipSuccess || hipEventCreate(&m->t1[i]) != hipSuccess)
                return CQ_ERR_HIP;
    }
    m->tune_step = 0;
    m->tune_len = most * reps;
    drop_graphs(m);  // partitions will change
    return CQ_OK;
}

int cq_multi_set_graph(cq_multi *m, int32_t on) {
    if (!m || (on != 0 && on != 1)) return CQ_ERR_INVALID;
    DeviceGuard guard(m->device);
    if (on) {
        for (cq_query *q : m->qs)
            if (!cq::query_capturable(q)) return CQ_ERR_INVALID;
        if (!m->origin && hipStreamCreateWithFlags(&m->origin, hipStreamNonBlocking) != hipSuccess)
            return CQ_ERR_HIP;
    } else {
        drop_graphs(m);
        for (cq_query *q : m->qs) (void)cq::query_set_graph(q, false, nullptr);
    }
    m->graph = on != 0;
    return CQ_OK;
}

int cq_multi_push(cq_multi *m, const int32_t *keys, const int32_t *values, int64_t n,
                  void *stream) {
    if (!m || n < 0 || n > CQ_MAX_BATCH || (n > 0 && (!keys || !values))) return CQ_ERR_INVALID;
    DeviceGuard guard(m->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool tuning = m->tune_step < m->tune_len;
    if (m->graph && !tuning) return graph_push(m, keys, values, n, s);
    int rc = enqueue_all(m, keys, values, n, s, tuning);
    if (rc != CQ_OK || !tuning) return rc;
    // tuning: collect this push's times (waits for it), advance the window
    const int nq = (int)m->qs.size();
    for (int i = 0; i < nq && rc == CQ_OK; ++i) {
        float ms = 0.f;
        rc = from_hip(hipEventSynchronize(m->t1[i]));
        if (rc == CQ_OK) rc = from_hip(hipEventElapsedTime(&ms, m->t0[i], m->t1[i]));
        if (rc == CQ_OK) m->times[i][cand_at(m, i, m->tune_step)].push_back(ms);
    }
    if (rc == CQ_OK && ++m->tune_step == m->tune_len) finish_tuning(m);
    return rc;
}

int cq_multi_plan(cq_multi *m, int32_t *modes, int32_t *workers, int32_t *lanes, float *ms) {
    if (!m) return CQ_ERR_INVALID;
    const int nq = (int)m->qs.size();
    const bool tuned = !m->chosen.empty() && m->tune_step >= m->tune_len;
    for (int i = 0; i < nq; ++i) {
        const Cand c = tuned ? m->cands[i][m->chosen[i]] : Cand{-1, -1};
        if (modes) modes[i] = c.mode;
        if (workers) workers[i] = c.workers;
        if (lanes) lanes[i] = m->lane_of[i];
        if (ms) ms[i] = tuned ? m->chosen_ms[i] : -1.f;
    }
    return CQ_OK;
}

int cq_multi_destroy(cq_multi *m) {
    if (!m) return CQ_OK;
    DeviceGuard guard(m->device);
    for (hipStream_t l : m->lanes) (void)hipStreamSynchronize(l);
    if (m->origin) (void)hipStreamSynchronize(m->origin);
    (void)hipDeviceSynchronize();  // replays run on the callers' streams
    drop_graphs(m);
    for (cq_query *q : m->qs) (void)cq::query_set_graph(q, false, nullptr);
    if (m->keys_st) (void)hipFree(m->keys_st);
    if (m->vals_st) (void)hipFree(m->vals_st);
    if (m->origin) (void)hipStreamDestroy(m->origin);
    for (hipStream_t l : m->lanes) (void)hipStreamDestroy(l);
    for (hipEvent_t j : m->joins) (void)hipEventDestroy(j);
    for (hipEvent_t t : m->t0) (void)hipEventDestroy(t);
    for (hipEvent_t t : m->t1) (void)hipEventDestroy(t);
    if (m->fork) (void)hipEventDestroy(m->fork);
    delete m;
    return CQ_OK;
}

}  // extern "C"
