// C-ABI runtime: query objects, device memory, per-batch launch sequence,
// telemetry.  See include/cq.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "cq.h"
#include "cq_balance.h"
#include "cq_internal.h"

using namespace cq;

namespace {

struct TimedLaunch {
    hipEvent_t start, stop;
    int kind;
};

}  // namespace

struct cq_query {
    int device = 0;
    uint32_t aggregates = 0;
    State st{};
    Scratch sc{};               // working buffers (batch-local arrays: set 0)
    Scratch alt{};              // second set of batch-local arrays (pipelined calls)
    bool have_alt = false;
    int cur = 0;                // set used by the most recent batch
    int mode = MODE_BALANCED;
    int32_t workers = 1024;
    int32_t seq = 0;            // batch sequence number (device-side epochs)
    int64_t last_n = 0;         // size of the most recent batch
    int last_mode = MODE_BALANCED;
    int32_t last_workers = 1024;
    hipStream_t last_stream = nullptr;
    bool pushed = false;
    int32_t telemetry = 0;
    int64_t trace_cap = 0;
    std::vector<TimedLaunch> live;
    std::vector<hipEvent_t> spare;
    double ms[CQ_KERNEL_KINDS] = {0};
    int64_t launches[CQ_KERNEL_KINDS] = {0};
    // Section 4 technique on the static workers (0: none)
    int policy = 0;
    Balancer bal;
    int32_t *m_owner = nullptr, *m_wstart = nullptr, *m_wlist = nullptr, *m_lidx = nullptr;
    int32_t *h_counts = nullptr;  // pinned: a batch's histogram, then its rejection flag
    int32_t *h_keys = nullptr;    // pinned: a sub-batch's keys (probCheck reads its tuples)
    int64_t h_keys_n = 0;         // keys in h_keys
    int32_t *h_map = nullptr;     // pinned: owner, wstart, wlist, lidx on their way up
    hipEvent_t ev_counts = nullptr, ev_map = nullptr;
    bool map_pending = false;     // an upload from h_map may still be running
    int64_t policy_total = 0;     // groups moved since the technique was selected
    uint64_t kmod = 0;            // keys reduced mod groups (multiplier; 0 = off)
    bool graph = false;           // pushes are being captured for replay
    // per-tuple results: arrival index of each staged tuple, count before
    // the sub-batch (allocated by the first per-tuple push)
    int32_t *pt_sidx = nullptr, *pt_pcnt = nullptr;
    // the last push was cq_push_batch_results_noalloc: its plan lives in the
    // shared scratch area, so cq_results / cq_status / cq_batch_plan refuse
    bool noalloc_last = false;
    // several batches per set of launches (allocated by the first such call)
    SbBufs sb{};
    bool have_sb = false;
};

namespace {

int from_hip(hipError_t e) {
    if (e == hipSuccess) return CQ_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return CQ_ERR_OOM;
    return CQ_ERR_HIP;
}

template <typename T>
int dalloc(T **p, int64_t count) {
    *p = nullptr;
    if (count < 1) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (size_t)count);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return from_hip(e);
    }
    return CQ_OK;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Makes the query's device current for the duration of a call.
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

// Batch-local arrays of one buffer set.
void free_set(Scratch &b) {
    dfree(b.k);
    dfree(b.lpre);
    dfree(b.bucket);
    dfree(b.pold);
    dfree(b.tidx);
    dfree(b.stamp);
    dfree(b.touched);
    dfree(b.ncnt);
    dfree(b.bstart);
    dfree(b.hkey);
    dfree(b.sdat);
    dfree(b.rowstart);
    dfree(b.partials);
    dfree(b.tot);
    dfree(b.bad);
}

// Allocates and clears the batch-local arrays of a set (histogram zero,
// plan totals zero); returns a status code.
int alloc_set(Scratch &b, int64_t G) {
    const int64_t nblk = (G + PLAN_CHUNK - 1) / PLAN_CHUNK;
    int rc = dalloc(&b.k, hist_entries(G));
    if (rc == CQ_OK) rc = dalloc(&b.lpre, G + 1);
    if (rc == CQ_OK) rc = dalloc(&b.bucket, G);
    if (rc == CQ_OK) rc = dalloc(&b.pold, G);
    if (rc == CQ_OK) rc = dalloc(&b.tidx, G);
    if (rc == CQ_OK) rc = dalloc(&b.stamp, G);
    if (rc == CQ_OK) rc = dalloc(&b.touched, G);
    if (rc == CQ_OK) rc = dalloc(&b.ncnt, G);
    if (rc == CQ_OK) rc = dalloc(&b.bstart, NB_MAX + 1);
    if (rc == CQ_OK) rc = dalloc(&b.hkey, NB_MAX);
    if (rc == CQ_OK) rc = dalloc(&b.sdat, SUB);
    if (rc == CQ_OK) rc = dalloc(&b.rowstart, (int64_t)PASS_TILES_MAX * (NB_MAX + 1));
    if (rc == CQ_OK) rc = dalloc(&b.partials, nblk * PLAN_FIELDS);
    if (rc == CQ_OK) rc = dalloc(&b.tot, 1);
    if (rc == CQ_OK) rc = dalloc(&b.bad, 1);
    if (rc != CQ_OK) return rc;
    hipError_t e = hipMemset(b.k, 0, sizeof(int32_t) * (size_t)hist_entries(G));
    if (e == hipSuccess) e = hipMemset(b.stamp, 0, sizeof(int32_t) * (size_t)G);
    if (e == hipSuccess) e = hipMemset(b.bucket, 0, sizeof(int32_t) * (size_t)G);
    if (e == hipSuccess) e = hipMemset(b.lpre, 0, sizeof(int32_t) * (size_t)(G + 1));
    if (e == hipSuccess) e = hipMemset(b.tot, 0, sizeof(PlanTotals));
    if (e == hipSuccess) e = hipMemset(b.bad, 0, sizeof(int32_t));
    return from_hip(e);
}

// Buffers of the several-batch path.
void free_sb(SbBufs &b) {
    dfree(b.kt);
    dfree(b.cut);
    dfree(b.kh);
    dfree(b.sbad);
    dfree(b.bucket);
    dfree(b.lpre);
    dfree(b.tidx);
    dfree(b.bstart);
    dfree(b.hkey);
    dfree(b.sdat);
    dfree(b.rowstart);
    dfree(b.tot);
    dfree(b.so);
    dfree(b.gsb);
    dfree(b.big);
    dfree(b.gbig);
    dfree(b.xs);
    dfree(b.ntot);
    dfree(b.tb);
    dfree(b.part);
}

int alloc_sb(SbBufs &b, int64_t G) {
    int rc = dalloc(&b.kh, G * SB_K);
    if (rc == CQ_OK) rc = dalloc(&b.kt, (int64_t)SB_K * SBH_TILES * ((G + 1) / 2));
    if (rc == CQ_OK) rc = dalloc(&b.cut, (int64_t)SB_K * G);
    if (rc == CQ_OK) rc = dalloc(&b.sbad, SB_K);
    if (rc == CQ_OK) rc = dalloc(&b.bucket, SB_K * G);
    if (rc == CQ_OK) rc = dalloc(&b.lpre, SB_K * (G + 1));
    if (rc == CQ_OK) rc = dalloc(&b.tidx, SB_K * G);
    if (rc == CQ_OK) rc = dalloc(&b.bstart, SB_K * (int64_t)(NB_MAX + 1));
    if (rc == CQ_OK) rc = dalloc(&b.hkey, SB_K * (int64_t)NB_MAX);
    if (rc == CQ_OK) rc = dalloc(&b.sdat, SB_K * (int64_t)SUB);
    if (rc == CQ_OK) rc = dalloc(&b.rowstart, SB_K * (int64_t)PASS_TILES_MAX * (NB_MAX + 1));
    if (rc == CQ_OK) rc = dalloc(&b.tot, SB_K);
    if (rc == CQ_OK) rc = dalloc(&b.so, SB_K * G);
    if (rc == CQ_OK) rc = dalloc(&b.gsb, G + 1);
    if (rc == CQ_OK) rc = dalloc(&b.big, G);
    if (rc == CQ_OK) rc = dalloc(&b.gbig, G);
    if (rc == CQ_OK) rc = dalloc(&b.xs, SB_K * (int64_t)SUB);
    if (rc == CQ_OK) rc = dalloc(&b.ntot, 2);
    if (rc == CQ_OK) rc = dalloc(&b.tb, SB_K * G);
    if (rc == CQ_OK) rc = dalloc(&b.part, (G + SBS_GROUPS - 1) / SBS_GROUPS * SBP_PART);
    if (rc != CQ_OK) return rc;
    hipError_t e = hipMemset(b.kh, 0, sizeof(int32_t) * (size_t)(G * SB_K));
    if (e == hipSuccess) e = hipMemset(b.sbad, 0, sizeof(int32_t) * SB_K);
    return from_hip(e);
}

void free_all(cq_query *q) {
    dfree(q->st.ring);
    dfree(q->st.pos);
    dfree(q->st.cnt);
    dfree(q->st.sum);
    free_set(q->sc);
    free_set(q->alt);
    dfree(q->sc.fault);
    dfree(q->sc.hot);
    dfree(q->sc.seqp);
    dfree(q->sc.trace);
    dfree(q->sc.phase);
    for (auto &t : q->live) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (auto e : q->spare) (void)hipEventDestroy(e);
    q->live.clear();
    q->spare.clear();
    dfree(q->m_owner);
    dfree(q->m_wstart);
    dfree(q->m_wlist);
    dfree(q->m_lidx);
    if (q->h_counts) (void)hipHostFree(q->h_counts);
    if (q->h_map) (void)hipHostFree(q->h_map);
    if (q->h_keys) (void)hipHostFree(q->h_keys);
    q->h_counts = q->h_map = q->h_keys = nullptr;
    if (q->ev_counts) (void)hipEventDestroy(q->ev_counts);
    if (q->ev_map) (void)hipEventDestroy(q->ev_map);
    q->ev_counts = q->ev_map = nullptr;
    dfree(q->pt_sidx);
    dfree(q->pt_pcnt);
    free_sb(q->sb);
    q->have_sb = false;
}

int ensure_trace(cq_query *q, int64_t records) {
    if (records <= q->trace_cap) return CQ_OK;
    dfree(q->sc.trace);
    int rc = dalloc(&q->sc.trace, 6 * records);
    if (rc != CQ_OK) {
        q->trace_cap = 0;
        return rc;
    }
    q->trace_cap = records;
    return CQ_OK;
}

hipEvent_t take_event(cq_query *q) {
    if (!q->spare.empty()) {
        hipEvent_t e = q->spare.back();
        q->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    // no system-scope fences: these events only time device work
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Launch one step, bracketed by events when kernel timing is on.
template <typename F>
int timed(cq_query *q, int kind, hipStream_t s, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (q->telemetry & CQ_TELEMETRY_KERNEL_TIMES) {
        a = take_event(q);
        b = take_event(q);
        if (a && b) (void)hipEventRecord(a, s);
    }
    hipError_t e = launch();
    if (a && b) {
        (void)hipEventRecord(b, s);
        q->live.push_back({a, b, kind});
    } else {
        if (a) q->spare.push_back(a);
        if (b) q->spare.push_back(b);
    }
    return from_hip(e);
}

bool static_ok(int64_t G, int32_t workers) {
    if (workers < 1 || workers > NB_MAX - 2) return false;
    return (G + workers - 1) / workers <= STATIC_KEYS_MAX;
}

// Buffer set i (batch-local arrays, key-check flag) with the shared ones
// (fault bits, hot groups, telemetry records; the records only when on).
Scratch set_of(const cq_query *q, int i) {
    Scratch b = i ? q->alt : q->sc;
    b.fault = q->sc.fault;
    b.hot = q->sc.hot;
    b.seqp = q->graph ? q->sc.seqp : nullptr;
    b.trace = (q->telemetry & CQ_TELEMETRY_WORKERS) ? q->sc.trace : nullptr;
    b.phase = (q->telemetry & CQ_TELEMETRY_PHASES) ? q->sc.phase : nullptr;
    b.kmod = q->kmod;
    const bool mapped = q->mode == MODE_STATIC && q->policy;
    b.owner = mapped ? q->m_owner : nullptr;
    b.wstart = mapped ? q->m_wstart : nullptr;
    b.wlist = mapped ? q->m_wlist : nullptr;
    b.lidx = mapped ? q->m_lidx : nullptr;
    return b;
}

// ---- Section 4 techniques: host-side mapping, one batch behind ----

// Device and pinned buffers of the mapping (once per query).
int policy_buffers(cq_query *q) {
    if (q->m_owner) return CQ_OK;
    const int64_t G = q->st.G;
    int rc = dalloc(&q->m_owner, G);
    if (rc == CQ_OK) rc = dalloc(&q->m_wstart, NB_MAX + 1);
    if (rc == CQ_OK) rc = dalloc(&q->m_wlist, G);
    if (rc == CQ_OK) rc = dalloc(&q->m_lidx, G);
    hipError_t e = hipSuccess;
    if (rc == CQ_OK)
        e = hipHostMalloc(reinterpret_cast<void **>(&q->h_counts), sizeof(int32_t) * (size_t)(G + 1),
                          hipHostMallocDefault);
    if (e == hipSuccess && rc == CQ_OK)
        e = hipHostMalloc(reinterpret_cast<void **>(&q->h_map),
                          sizeof(int32_t) * (size_t)(3 * G + NB_MAX + 1), hipHostMallocDefault);
    if (e == hipSuccess && rc == CQ_OK)
        e = hipHostMalloc(reinterpret_cast<void **>(&q->h_keys), sizeof(int32_t) * (size_t)SUB,
                          hipHostMallocDefault);
    if (e == hipSuccess && rc == CQ_OK)
        e = hipEventCreateWithFlags(&q->ev_counts, hipEventDisableTiming);
    if (e == hipSuccess && rc == CQ_OK) e = hipEventCreateWithFlags(&q->ev_map, hipEventDisableTiming);
    if (rc == CQ_OK) rc = from_hip(e);
    if (rc != CQ_OK) {
        dfree(q->m_owner);
        dfree(q->m_wstart);
        dfree(q->m_wlist);
        dfree(q->m_lidx);
        if (q->h_counts) (void)hipHostFree(q->h_counts);
        if (q->h_map) (void)hipHostFree(q->h_map);
        if (q->h_keys) (void)hipHostFree(q->h_keys);
        q->h_counts = q->h_map = q->h_keys = nullptr;
        if (q->ev_counts) (void)hipEventDestroy(q->ev_counts);
        if (q->ev_map) (void)hipEventDestroy(q->ev_map);
        q->ev_counts = q->ev_map = nullptr;
    }
    return rc;
}

// Enqueues the upload of the balancer's mapping on s (after the work
// already on s, before whatever is enqueued next).
int policy_upload(cq_query *q, hipStream_t s) {
    const int64_t G = q->st.G;
    const int32_t T = q->bal.T;
    if (q->map_pending && hipEventSynchronize(q->ev_map) != hipSuccess) return CQ_ERR_HIP;
    int32_t *owner = q->h_map, *wstart = owner + G, *wlist = wstart + T + 1, *lidx = wlist + G;
    std::copy(q->bal.owner.begin(), q->bal.owner.end(), owner);
    q->bal.export_csr(wstart, wlist, lidx);
    const size_t gb = sizeof(int32_t) * (size_t)G;
    hipError_t e = hipMemcpyAsync(q->m_owner, owner, gb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(q->m_wstart, wstart, sizeof(int32_t) * (size_t)(T + 1),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(q->m_wlist, wlist, gb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(q->m_lidx, lidx, gb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(q->ev_map, s);
    q->map_pending = e == hipSuccess;
    return from_hip(e);
}

// After the histogram of a (sub-)batch of m tuples: its counts and
// rejection flag on their way to the host, and under probCheck its keys
// too (the technique reads the most loaded worker's tuples in arrival
// order).
int policy_fetch(cq_query *q, const Scratch &sc, const int32_t *keys, int64_t m,
                 hipStream_t s) {
    const int64_t G = q->st.G;
    hipError_t e = hipMemcpyAsync(q->h_counts, sc.k, sizeof(int32_t) * (size_t)G,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(q->h_counts + G, sc.bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    q->h_keys_n = 0;
    if (e == hipSuccess && q->policy == CQ_PARTITION_PROBCHECK && m > 0) {
        e = hipMemcpyAsync(q->h_keys, keys, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost, s);
        q->h_keys_n = m;
    }
    if (e == hipSuccess) e = hipEventRecord(q->ev_counts, s);
    return from_hip(e);
}

// After the rest of the batch is enqueued: wait for its counts, run one
// step of the technique, and send a changed mapping up for the next batch.
int policy_step(cq_query *q, int32_t seq, hipStream_t s) {
    if (hipEventSynchronize(q->ev_counts) != hipSuccess) return CQ_ERR_HIP;
    q->bal.last_moves = 0;
    if (q->h_counts[q->st.G] == seq) return CQ_OK;  // rejected batch: nothing happened
    if (q->kmod && q->h_keys_n > 0) {  // the groups the query sees
        const uint32_t G = (uint32_t)q->st.G;
        for (int64_t i = 0; i < q->h_keys_n; ++i)
            q->h_keys[i] = (int32_t)((uint32_t)q->h_keys[i] % G);
    }
    const int64_t moved = q->bal.step(q->policy, q->h_counts, q->h_keys, q->h_keys_n);
    q->policy_total += moved;
    return moved ? policy_upload(q, s) : CQ_OK;
}

// Telemetry buffers for sub-batches of up to n tuples.
int prepare_telemetry(cq_query *q, int64_t n) {
    if (q->telemetry & CQ_TELEMETRY_WORKERS) {
        const int64_t grid =
            update_grid(std::min<int64_t>(std::max<int64_t>(n, 1), SUB), q->mode, q->workers);
        const int rc = ensure_trace(q, grid);
        if (rc != CQ_OK) return rc;
    }
    if ((q->telemetry & CQ_TELEMETRY_PHASES) && !q->sc.phase) {
        const int rc = dalloc(&q->sc.phase, (int64_t)PHASE_KINDS * PHASE_BLOCKS * PHASE_SLOTS);
        if (rc != CQ_OK) return rc;
        (void)hipMemset(q->sc.phase, 0,
                        sizeof(int64_t) * (size_t)PHASE_KINDS * PHASE_BLOCKS * PHASE_SLOTS);
    }
    return CQ_OK;
}

// Histogram (unless already enqueued), plan and reorder of one sub-batch.
int front(cq_query *q, const int32_t *keys, const int32_t *values, int64_t m, const Scratch &sc,
          int32_t seq, hipStream_t s, bool have_hist = false) {
    int rc = CQ_OK;
    if (!have_hist)
        rc = timed(q, CQ_KERNEL_HIST, s,
                   [&] { return launch_hist(keys, m, q->st.G, sc, seq, s); });
    if (rc == CQ_OK && sc.owner) rc = policy_fetch(q, sc, keys, m, s);
    if (rc == CQ_OK && !plan_fused(q->st.G))
        rc = timed(q, CQ_KERNEL_PLAN, s,
                   [&] { return launch_plan(q->st, sc, seq, q->mode, q->workers, s); });
    if (rc == CQ_OK)
        rc = timed(q, CQ_KERNEL_PASS, s, [&] {
            return launch_pass(keys, values, m, q->st, sc, seq, q->mode, q->workers, s);
        });
    return rc;
}

// The whole per-batch sequence; `out` non-null means emit into it.
int push(cq_query *q, const int32_t *keys, const int32_t *values, int64_t n, hipStream_t s,
         const Out *out, const PtOut *pt = nullptr) {
    if (q->mode == MODE_STATIC && !static_ok(q->st.G, q->workers)) return CQ_ERR_INVALID;
    const int64_t nsub = (n + SUB - 1) / SUB;
    int rc = prepare_telemetry(q, n);
    if (rc != CQ_OK) return rc;
    q->cur = 0;
    Scratch sc = set_of(q, 0);
    if (pt) {
        sc.sidx = q->pt_sidx;
        sc.pcnt = q->pt_pcnt;
    }
    if (sc.owner && q->map_pending && hipStreamWaitEvent(s, q->ev_map, 0) != hipSuccess)
        return CQ_ERR_HIP;
    q->last_stream = s;
    q->pushed = true;
    q->noalloc_last = false;
    q->last_n = n;
    q->last_mode = q->mode;
    q->last_workers = q->workers;
    const int32_t seq = ++q->seq;
    if (sc.seqp) {  // captured: the replayed push advances its own number
        rc = from_hip(launch_bump_seq(sc, s));
        if (rc != CQ_OK) {
            --q->seq;
            return rc;
        }
    }
    if (n == 0) {
        rc = from_hip(launch_reset_totals(sc, s));
        if (rc == CQ_OK && out)
            rc = timed(q, CQ_KERNEL_EMIT, s, [&] { return launch_emit(q->st, sc, 1, *out, s); });
        return rc;
    }
    const int64_t G = q->st.G;
    if (nsub > 1)
        rc = timed(q, CQ_KERNEL_OTHER, s,
                   [&] { return launch_validate(keys, n, G, seq, sc, s); });
    const Out none = {nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int64_t b = 0; b < nsub && rc == CQ_OK; ++b) {
        const int64_t off = b * SUB;
        const int64_t m = std::min<int64_t>(SUB, n - off);
        const Out o = (out && nsub == 1) ? *out : none;
        rc = front(q, keys + off, values + off, m, sc, seq, s);
        if (rc == CQ_OK && pt) {
            PtOut po = *pt;  // this sub-batch's tuples
            if (po.sums) po.sums += off;
            if (po.counts) po.counts += off;
            if (po.avgs) po.avgs += off;
            rc = timed(q, CQ_KERNEL_TUPLES, s, [&] { return launch_tuples(q->st, sc, m, po, s); });
        }
        if (rc == CQ_OK)
            rc = timed(q, CQ_KERNEL_UPDATE, s, [&] {
                return launch_update(q->st, sc, m, q->mode, q->workers, o, s);
            });
        if (rc == CQ_OK && sc.owner) rc = policy_step(q, seq, s);
    }
    if (rc == CQ_OK && nsub > 1) {
        rc = timed(q, CQ_KERNEL_OTHER, s,
                   [&] { return launch_collect_touched(G, seq, sc, s); });
        if (rc == CQ_OK && out) {
            const int64_t cap = std::min<int64_t>(G, n);
            rc = timed(q, CQ_KERNEL_EMIT, s,
                       [&] { return launch_emit(q->st, sc, cap, *out, s); });
        }
    }
    return rc;
}

// Second buffer set (first pipelined call).
int ensure_alt(cq_query *q) {
    if (q->have_alt) return CQ_OK;
    int rc = alloc_set(q->alt, q->st.G);
    if (rc == CQ_OK) rc = from_hip(hipDeviceSynchronize());
    if (rc != CQ_OK) {
        free_set(q->alt);
        return rc;
    }
    q->have_alt = true;
    return CQ_OK;
}

// Whether cq_push_batches takes the several-batch path: up to PASS_LOCAL_G
// groups, the balanced partition, no technique, no capture, no per-workgroup
// records (kernel times and phase clocks are recorded).
bool sb_eligible(const cq_query *q) {
    return q->st.G <= PASS_LOCAL_G && q->mode == MODE_BALANCED && !q->policy && !q->graph &&
           !(q->telemetry & CQ_TELEMETRY_WORKERS);
}

int ensure_sb(cq_query *q) {
    if (q->have_sb) return CQ_OK;
    int rc = alloc_sb(q->sb, q->st.G);
    if (rc == CQ_OK) rc = from_hip(hipDeviceSynchronize());
    if (rc != CQ_OK) {
        free_sb(q->sb);
        return rc;
    }
    q->have_sb = true;
    return CQ_OK;
}

// cq_push_batches in groups of up to SB_K batches, six launches each; a
// longer call is cut into ceil(count / SB_K) groups of near-equal size, so
// that no group is left with a few batches to carry a whole chain's fixed
// cost.
int push_sb(cq_query *q, int32_t count, const int32_t *const *keys,
            const int32_t *const *values, const int64_t *n, int32_t *const *ids,
            int64_t *const *sums, int32_t *const *counts, double *const *avgs,
            int64_t *const *n_touched, hipStream_t s) {
    int rc = ensure_sb(q);
    if (rc == CQ_OK) rc = prepare_telemetry(q, SUB);
    if (rc != CQ_OK) return rc;
    const Scratch base = set_of(q, 0);
    q->sb.fault = q->sc.fault;
    const int32_t chains = (count + SB_K - 1) / SB_K;
    for (int32_t c = 0, c0 = 0; c < chains && rc == CQ_OK; ++c) {
        SbBatches in{};
        in.K = count / chains + (c < count % chains ? 1 : 0);
        int32_t ht = 0, pt = 0;
        for (int b = 0; b < in.K; ++b) {
            const int32_t i = c0 + b;
            in.keys[b] = keys[i];
            in.values[b] = values[i];
            in.n[b] = n[i];
            in.htile0[b] = ht;
            in.ptile0[b] = pt;
            ht += (int32_t)((n[i] + SBH_TILE - 1) / SBH_TILE);
            pt += (int32_t)((n[i] + PASS_TILE - 1) / PASS_TILE);
            if (((uintptr_t)keys[i] & 15u) == 0) in.vec |= 1u << b;
            in.out[b] = {ids ? ids[i] : nullptr, sums ? sums[i] : nullptr,
                         counts ? counts[i] : nullptr, avgs ? avgs[i] : nullptr, n_touched[i]};
        }
        in.htile0[in.K] = ht;
        in.ptile0[in.K] = pt;
        const int32_t seq = ++q->seq;
        rc = timed(q, CQ_KERNEL_HIST, s, [&] { return launch_sb_hist(q->st, base, q->sb, in, seq, s); });
        if (rc == CQ_OK)
            rc = timed(q, CQ_KERNEL_PLAN, s,
                       [&] { return launch_sb_plan(q->st, base, q->sb, in, seq, s); });
        if (rc == CQ_OK)
            rc = timed(q, CQ_KERNEL_PASS, s,
                       [&] { return launch_sb_pass(q->st, base, q->sb, in, seq, s); });
        if (rc == CQ_OK)
            rc = timed(q, CQ_KERNEL_PREP, s,
                       [&] { return launch_sb_prep(q->st, base, q->sb, in, s); });
        if (rc == CQ_OK)
            rc = timed(q, CQ_KERNEL_APPLY, s,
                       [&] { return launch_sb_apply(q->st, base, q->sb, in, seq, s); });
        c0 += in.K;
    }
    // cq_results, cq_status and cq_batch_plan read the last batch's plan,
    // which the several-batch plan also leaves in buffer set 0
    q->cur = 0;
    q->last_n = n[count - 1];
    q->last_stream = s;
    q->pushed = true;
    q->noalloc_last = false;
    q->last_mode = q->mode;
    q->last_workers = q->workers;
    return rc;
}

}  // namespace

namespace cq {

// Whether a query's pushes can be captured into a graph: no host step
// (techniques), no telemetry events, no per-tuple outputs.
bool query_capturable(const cq_query *q) { return !q->policy && !q->telemetry; }

// Enters or leaves capture mode.  Entering sets the device copy of the
// sequence number to the host's (on stream s, before the capture starts).
int query_set_graph(cq_query *q, bool on, hipStream_t s) {
    DeviceGuard guard(q->device);
    if (on && !q->graph) {
        q->graph = true;
        const int rc = from_hip(launch_set_seq(set_of(q, 0), q->seq, s));
        if (rc != CQ_OK) q->graph = false;
        return rc;
    }
    q->graph = on;
    return CQ_OK;
}

// The stream a query's last work was enqueued on (captured pushes run
// where their graph is launched).
void query_ran_on(cq_query *q, hipStream_t s) { q->last_stream = s; }

// After a replay of a captured push of n tuples on stream s: the host's
// record of the query follows what the replay did on the device.
void query_replayed(cq_query *q, int64_t n, hipStream_t s) {
    q->seq += 1;
    q->cur = 0;
    q->last_n = n;
    q->last_stream = s;
    q->pushed = true;
    q->last_mode = q->mode;
    q->last_workers = q->workers;
}

}  // namespace cq

extern "C" {

const char *cq_strerror(int code) {
    switch (code) {
        case CQ_OK: return "success";
        case CQ_ERR_INVALID: return "invalid argument";
        case CQ_ERR_OOM: return "out of device memory";
        case CQ_ERR_KEY_RANGE: return "batch rejected: key outside [0, groups)";
        case CQ_ERR_HIP: return "HIP runtime error";
        default: return "unknown status code";
    }
}

int cq_create(int64_t groups, int32_t window, uint32_t aggregates, cq_query **out) {
    if (!out) return CQ_ERR_INVALID;
    *out = nullptr;
    if (groups < 1 || groups > INT32_MAX - 1 || window < 1 || window > CQ_MAX_WINDOW)
        return CQ_ERR_INVALID;
    if (aggregates == 0 || (aggregates & ~(CQ_SUM | CQ_COUNT | CQ_AVG)) != 0)
        return CQ_ERR_INVALID;
    cq_query *q = new (std::nothrow) cq_query();
    if (!q) return CQ_ERR_OOM;
    if (hipGetDevice(&q->device) != hipSuccess) {
        delete q;
        return CQ_ERR_HIP;
    }
    q->aggregates = aggregates;
    q->st.G = groups;
    q->st.W = window;
    const int64_t G = groups;
    int rc = dalloc(&q->st.ring, G * (int64_t)window);
    if (rc == CQ_OK) rc = dalloc(&q->st.pos, G);
    if (rc == CQ_OK) rc = dalloc(&q->st.cnt, G);
    if (rc == CQ_OK) rc = dalloc(&q->st.sum, G);
    if (rc == CQ_OK) rc = alloc_set(q->sc, G);
    if (rc == CQ_OK) rc = dalloc(&q->sc.fault, 1);
    if (rc == CQ_OK) rc = dalloc(&q->sc.hot, 2);
    if (rc == CQ_OK) rc = dalloc(&q->sc.seqp, 1);
    hipError_t e = hipSuccess;
    if (rc == CQ_OK) {
        // zero-filled windows: never-written slots read as 0, so the first
        // W insertions of a group subtract nothing
        e = hipMemset(q->st.ring, 0, sizeof(int32_t) * (size_t)(G * (int64_t)window));
        if (e == hipSuccess) e = hipMemset(q->st.pos, 0, sizeof(int32_t) * (size_t)G);
        if (e == hipSuccess) e = hipMemset(q->st.cnt, 0, sizeof(int32_t) * (size_t)G);
        if (e == hipSuccess) e = hipMemset(q->st.sum, 0, sizeof(int64_t) * (size_t)G);
        if (e == hipSuccess) e = hipMemset(q->sc.fault, 0, sizeof(int32_t));
        if (e == hipSuccess) e = hipMemset(q->sc.hot, 0xff, 2 * sizeof(int32_t));
        if (e == hipSuccess) e = hipMemset(q->sc.seqp, 0, sizeof(int32_t));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        rc = from_hip(e);
    }
    if (rc != CQ_OK) {
        free_all(q);
        delete q;
        return rc;
    }
    *out = q;
    return CQ_OK;
}

int64_t cq_query_footprint(int64_t groups, int32_t window) {
    if (groups < 1 || groups > INT32_MAX - 1 || window < 1 || window > CQ_MAX_WINDOW) return -1;
    const int64_t G = groups;
    auto pg = [](int64_t bytes) { return (std::max<int64_t>(bytes, 1) + 4095) / 4096 * 4096; };
    const int64_t nblk = (G + PLAN_CHUNK - 1) / PLAN_CHUNK;
    int64_t b = pg(4 * G * (int64_t)window) + 2 * pg(4 * G) + pg(8 * G);  // ring, pos, cnt, sum
    b += pg(4 * hist_entries(G)) + 6 * pg(4 * G) + pg(4 * (G + 1));       // histogram, per-group plan
    b += pg(4 * (NB_MAX + 1)) + pg(4 * NB_MAX);                          // bucket starts, heavy keys
    b += pg(8 * (int64_t)SUB) + pg(4 * (int64_t)PASS_TILES_MAX * (NB_MAX + 1));  // staging, runs
    b += pg(4 * nblk * PLAN_FIELDS) + pg(sizeof(PlanTotals)) + pg(4) + pg(4) + pg(8);
    return b;
}

int cq_reserve(cq_query *q, int64_t max_batch) {
    // every working buffer is sized at cq_create (batches are processed in
    // fixed-size sub-batches), so there is nothing left to reserve
    if (!q || max_batch < 0 || max_batch > CQ_MAX_BATCH) return CQ_ERR_INVALID;
    return CQ_OK;
}

int cq_set_partition(cq_query *q, int32_t mode, int32_t workers) {
    if (!q) return CQ_ERR_INVALID;
    if (mode < CQ_PARTITION_BALANCED || mode > CQ_PARTITION_SHIFTLOCAL) return CQ_ERR_INVALID;
    if (workers < 0) return CQ_ERR_INVALID;
    const int32_t w = workers ? workers : 1024;
    if (mode != CQ_PARTITION_BALANCED && !static_ok(q->st.G, w)) return CQ_ERR_INVALID;
    const bool technique = mode >= CQ_PARTITION_GETFIRST;
    if (technique) {
        DeviceGuard guard(q->device);
        int rc = policy_buffers(q);
        if (rc != CQ_OK) return rc;
        // the device mapping may still be read by pushes in flight
        if (hipDeviceSynchronize() != hipSuccess) return CQ_ERR_HIP;
        q->bal.reset(w, q->st.G);
        q->bal.max_keys = STATIC_KEYS_MAX;
        q->bal.last_moves = q->bal.last_max = q->bal.last_min = 0;
        q->policy_total = 0;
        rc = policy_upload(q, nullptr);
        if (rc == CQ_OK && hipEventSynchronize(q->ev_map) != hipSuccess) rc = CQ_ERR_HIP;
        q->map_pending = false;
        if (rc != CQ_OK) return rc;
    }
    q->policy = technique ? mode : 0;
    q->mode = mode == CQ_PARTITION_BALANCED ? MODE_BALANCED : MODE_STATIC;
    q->workers = w;
    return CQ_OK;
}

int cq_query_groups(const cq_query *q, int64_t *groups) {
    if (!q || !groups) return CQ_ERR_INVALID;
    *groups = q->st.G;
    return CQ_OK;
}

int cq_set_key_mod(cq_query *q, int32_t on) {
    if (!q || (on != 0 && on != 1)) return CQ_ERR_INVALID;
    const uint64_t G = (uint64_t)q->st.G;
    q->kmod = on ? (G == 1 ? 1 : UINT64_MAX / G + 1) : 0;
    return CQ_OK;
}

int cq_set_policy_params(cq_query *q, int64_t threshold, double pot) {
    if (!q || threshold < 0 || !(pot > 0.0 && pot <= 1.0)) return CQ_ERR_INVALID;
    q->bal.threshold = threshold;
    q->bal.pot = pot;
    return CQ_OK;
}

int cq_policy_stats(cq_query *q, int64_t *out) {
    if (!q || !out) return CQ_ERR_INVALID;
    const bool on = q->policy != 0;
    out[0] = on ? q->bal.last_moves : 0;
    out[1] = on ? q->bal.last_max : 0;
    out[2] = on ? q->bal.last_min : 0;
    out[3] = on ? q->policy_total : 0;
    return CQ_OK;
}

int cq_push_batch(cq_query *q, const int32_t *keys, const int32_t *values, int64_t n,
                  void *stream) {
    if (!q || n < 0 || n > CQ_MAX_BATCH) return CQ_ERR_INVALID;
    if (n > 0 && (!keys || !values)) return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    return push(q, keys, values, n, reinterpret_cast<hipStream_t>(stream), nullptr);
}

int cq_push_batch_results(cq_query *q, const int32_t *keys, const int32_t *values, int64_t n,
                          int32_t *ids, int64_t *sums, int32_t *counts, double *avgs,
                          int64_t *n_touched, void *stream) {
    if (!q || n < 0 || n > CQ_MAX_BATCH || !n_touched) return CQ_ERR_INVALID;
    if (n > 0 && (!keys || !values)) return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    const Out out = {ids, sums, counts, avgs, n_touched};
    return push(q, keys, values, n, reinterpret_cast<hipStream_t>(stream), &out);
}

int cq_push_batch_results_noalloc(cq_query *q, const int32_t *keys, const int32_t *values,
                                  int64_t n, int32_t *ids, int64_t *sums, int32_t *counts,
                                  double *avgs, int64_t *n_touched, void *stream) {
    if (!q || n < 0 || n > CQ_NOALLOC_MAX_BATCH || !n_touched) return CQ_ERR_INVALID;
    if (n > 0 && (!keys || !values)) return CQ_ERR_INVALID;
    if (q->st.G > CQ_NOALLOC_MAX_GROUPS || q->mode != MODE_BALANCED || q->policy)
        return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    char *base = noalloc_base(q->device);
    if (!base) return CQ_ERR_HIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Scratch sc = noalloc_set(base);
    sc.fault = q->sc.fault;
    sc.hot = q->sc.hot;
    sc.kmod = q->kmod;
    q->last_stream = s;
    q->pushed = true;
    q->noalloc_last = true;
    q->last_n = n;
    if (n == 0) return from_hip(launch_set_touched(n_touched, 0, s));
    // The scratch area keeps whatever the previous call on this device left:
    // the histogram and the bad-key flag are cleared first, and the flag's
    // batch number is the constant 1, so a replayed capture stays valid.
    const int32_t seq = 1;
    const Out out = {ids, sums, counts, avgs, n_touched};
    hipError_t e = launch_noalloc_clear(sc, s);
    if (e == hipSuccess) e = launch_hist(keys, n, q->st.G, sc, seq, s);
    if (e == hipSuccess) e = launch_pass(keys, values, n, q->st, sc, seq, MODE_BALANCED, 0, s);
    if (e == hipSuccess) e = launch_update(q->st, sc, n, MODE_BALANCED, 0, out, s);
    return from_hip(e);
}

int cq_push_batch_tuples(cq_query *q, const int32_t *keys, const int32_t *values, int64_t n,
                         int32_t passes, int64_t *sums, int32_t *counts, double *avgs,
                         void *stream) {
    if (!q || n < 0 || n > CQ_MAX_BATCH || passes < 0 || passes > CQ_TUPLE_MAX_PASSES)
        return CQ_ERR_INVALID;
    if (n > 0 && (!keys || !values)) return CQ_ERR_INVALID;
    if (q->mode != MODE_BALANCED || q->st.G > CQ_TUPLE_MAX_GROUPS || q->st.W > CQ_TUPLE_MAX_WINDOW)
        return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    if (!q->pt_sidx) {
        int rc = dalloc(&q->pt_sidx, SUB);
        if (rc == CQ_OK) rc = dalloc(&q->pt_pcnt, q->st.G);
        if (rc != CQ_OK) {
            dfree(q->pt_sidx);
            dfree(q->pt_pcnt);
            return rc;
        }
    }
    const PtOut pt = {sums, counts, avgs, passes};
    return push(q, keys, values, n, reinterpret_cast<hipStream_t>(stream), nullptr, &pt);
}

int cq_push_batches(cq_query *q, int32_t count, const int32_t *const *keys,
                    const int32_t *const *values, const int64_t *n, int32_t *const *ids,
                    int64_t *const *sums, int32_t *const *counts, double *const *avgs,
                    int64_t *const *n_touched, void *stream) {
    if (!q || count < 0) return CQ_ERR_INVALID;
    if (count == 0) return CQ_OK;
    if (!keys || !values || !n || !n_touched) return CQ_ERR_INVALID;
    for (int32_t i = 0; i < count; ++i) {
        if (n[i] < 0 || n[i] > SUB || !n_touched[i]) return CQ_ERR_INVALID;
        if (n[i] > 0 && (!keys[i] || !values[i])) return CQ_ERR_INVALID;
    }
    if (q->mode == MODE_STATIC && !static_ok(q->st.G, q->workers)) return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    if (sb_eligible(q))
        return push_sb(q, count, keys, values, n, ids, sums, counts, avgs, n_touched,
                       reinterpret_cast<hipStream_t>(stream));
    int rc = ensure_alt(q);
    if (rc == CQ_OK) rc = prepare_telemetry(q, SUB);
    if (rc != CQ_OK) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool mapped = q->mode == MODE_STATIC && q->policy;
    if (mapped && q->map_pending && hipStreamWaitEvent(s, q->ev_map, 0) != hipSuccess)
        return CQ_ERR_HIP;
    const int32_t seq0 = q->seq + 1;
    q->seq += count;
    q->noalloc_last = false;
    // Batch i uses buffer set i mod 2.  Batch i+1's histogram is computed
    // by extra workgroups of batch i's update launch (it only needs its own
    // set's histogram, cleared by batch i-1's update), so a batch costs two
    // launches instead of three; everything stays on the caller's stream.
    bool have_hist = false;
    for (int32_t i = 0; i < count && rc == CQ_OK; ++i) {
        const int b = i & 1;
        const Scratch sc = set_of(q, b);
        const int32_t seq = seq0 + i;
        const Out out = {ids ? ids[i] : nullptr, sums ? sums[i] : nullptr,
                         counts ? counts[i] : nullptr, avgs ? avgs[i] : nullptr, n_touched[i]};
        q->cur = b;
        q->last_n = n[i];
        if (sc.seqp) {  // captured: the replayed push advances its own number
            rc = from_hip(launch_bump_seq(sc, s));
            if (rc != CQ_OK) {
                q->seq = seq - 1;  // the batches from here on never reached the device
                break;
            }
        }
        if (n[i] == 0) {
            rc = from_hip(launch_reset_totals(sc, s));
            if (rc == CQ_OK) rc = from_hip(launch_set_touched(n_touched[i], 0, s));
            have_hist = false;
            continue;
        }
        rc = front(q, keys[i], values[i], n[i], sc, seq, s, have_hist);
        const bool fuse =
            i + 1 < count && n[i + 1] > 0 && !mapped && can_fuse_hist(q->st.G, q->mode);
        if (rc == CQ_OK)
            rc = timed(q, CQ_KERNEL_UPDATE, s, [&] {
                return fuse ? launch_update(q->st, sc, n[i], q->mode, q->workers, out, s,
                                            keys[i + 1], n[i + 1], set_of(q, (i + 1) & 1),
                                            seq + 1)
                            : launch_update(q->st, sc, n[i], q->mode, q->workers, out, s);
            });
        if (rc == CQ_OK && mapped) rc = policy_step(q, seq, s);
        have_hist = fuse;
    }
    q->last_stream = s;
    q->pushed = true;
    q->last_mode = q->mode;
    q->last_workers = q->workers;
    return rc;
}

int cq_results(cq_query *q, int32_t *ids, int64_t *sums, int32_t *counts, double *avgs,
               int64_t *n_touched, void *stream) {
    if (!q || !n_touched || q->noalloc_last) return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t cap = std::min<int64_t>(q->st.G, q->last_n);
    const Out out = {ids, sums, counts, avgs, n_touched};
    const Scratch sc = set_of(q, q->cur);
    int rc = timed(q, CQ_KERNEL_EMIT, s, [&] { return launch_emit(q->st, sc, cap, out, s); });
    q->last_stream = s;
    q->pushed = true;
    return rc;
}

int cq_status(cq_query *q) {
    if (!q || q->noalloc_last) return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    hipError_t e = hipStreamSynchronize(q->last_stream);
    if (e != hipSuccess) return from_hip(e);
    PlanTotals t;
    e = hipMemcpy(&t, set_of(q, q->cur).tot, sizeof(t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return from_hip(e);
    return t.status;
}

int cq_destroy(cq_query *q) {
    if (!q) return CQ_OK;
    DeviceGuard guard(q->device);
    int rc = CQ_OK;
    if (q->pushed) rc = from_hip(hipStreamSynchronize(q->last_stream));
    free_all(q);
    delete q;
    return rc;
}

int cq_set_telemetry(cq_query *q, int32_t flags) {
    if (!q || (flags & ~(CQ_TELEMETRY_KERNEL_TIMES | CQ_TELEMETRY_WORKERS |
                         CQ_TELEMETRY_PHASES)) != 0)
        return CQ_ERR_INVALID;
    q->telemetry = flags;
    return CQ_OK;
}

int cq_kernel_times(cq_query *q, double *ms, int64_t *launches, int32_t nkinds) {
    if (!q || nkinds < 0 || (nkinds > 0 && (!ms || !launches))) return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    int rc = CQ_OK;
    for (auto &t : q->live) {
        hipError_t e = hipEventSynchronize(t.stop);
        float el = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&el, t.start, t.stop);
        if (e != hipSuccess) {
            rc = from_hip(e);
        } else {
            q->ms[t.kind] += el;
            q->launches[t.kind] += 1;
        }
        q->spare.push_back(t.start);
        q->spare.push_back(t.stop);
    }
    q->live.clear();
    for (int k = 0; k < nkinds && k < CQ_KERNEL_KINDS; ++k) {
        ms[k] = q->ms[k];
        launches[k] = q->launches[k];
    }
    for (int k = 0; k < CQ_KERNEL_KINDS; ++k) {
        q->ms[k] = 0;
        q->launches[k] = 0;
    }
    return rc;
}

int cq_worker_trace(cq_query *q, int64_t *rec, int64_t cap, int64_t *count) {
    if (!q || !count || cap < 0 || (cap > 0 && !rec)) return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    *count = 0;
    if (!(q->telemetry & CQ_TELEMETRY_WORKERS) || !q->sc.trace || q->last_n == 0) return CQ_OK;
    hipError_t e = hipStreamSynchronize(q->last_stream);
    if (e != hipSuccess) return from_hip(e);
    const int64_t have = std::min(
        q->trace_cap,
        update_grid(std::min<int64_t>(q->last_n, SUB), q->last_mode, q->last_workers));
    *count = have;
    const int64_t m = std::min(have, cap);
    if (m > 0) {
        e = hipMemcpy(rec, q->sc.trace, sizeof(int64_t) * 6 * (size_t)m, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return from_hip(e);
    }
    return CQ_OK;
}

int cq_phase_trace(cq_query *q, int32_t kind, int64_t *out, int64_t cap, int64_t *count) {
    if (!q || !count || kind < 0 || kind >= PHASE_KINDS || cap < 0 || (cap > 0 && !out))
        return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    *count = 0;
    if (!(q->telemetry & CQ_TELEMETRY_PHASES) || !q->sc.phase) return CQ_OK;
    hipError_t e = hipStreamSynchronize(q->last_stream);
    if (e != hipSuccess) return from_hip(e);
    *count = PHASE_BLOCKS;
    const int64_t m = std::min<int64_t>(PHASE_BLOCKS, cap);
    if (m > 0) {
        e = hipMemcpy(out, q->sc.phase + (int64_t)kind * PHASE_BLOCKS * PHASE_SLOTS,
                      sizeof(int64_t) * PHASE_SLOTS * (size_t)m, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return from_hip(e);
    }
    return CQ_OK;
}

int cq_batch_plan(cq_query *q, int64_t *out) {
    if (!q || !out || q->noalloc_last) return CQ_ERR_INVALID;
    DeviceGuard guard(q->device);
    hipError_t e = hipStreamSynchronize(q->last_stream);
    if (e != hipSuccess) return from_hip(e);
    PlanTotals t;
    e = hipMemcpy(&t, set_of(q, q->cur).tot, sizeof(t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return from_hip(e);
    int32_t fault = 0;
    e = hipMemcpy(&fault, q->sc.fault, sizeof(fault), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return from_hip(e);
    out[0] = t.n_light_buckets;
    out[1] = t.n_heavy;
    out[2] = t.light_tuples;
    out[3] = t.n_touched;
    out[4] = t.n_buckets;
    out[5] = t.sub_touched;
    out[6] = t.status;
    out[7] = (std::min<int64_t>(q->last_n, SUB) + PASS_TILE - 1) / PASS_TILE;
    out[8] = fault;
    return CQ_OK;
}

}  // extern "C"
