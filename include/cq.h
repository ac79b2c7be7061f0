/*
 * cq.h -- continuous sliding-window group-by aggregation on MI355X (gfx950).
 *
 * One query maintains, for every group id g in [0, groups), a count window
 * holding the last `window` integer values seen for g, and its SUM, COUNT
 * and AVG.  Tuples arrive in batches of (key, value) int32 pairs.  This is
 * the continuous aggregate query of Koutsoumpakis, Koutsoumpakis and
 * Gounaris, "Skew Handling in Aggregate Streaming Queries on GPUs" (ADMS
 * 2013): tuples are (group identifier id, integer attr) pairs and the
 * aggregate of a group depends on the last values received for it under a
 * fixed-size window (Section 3, problem statement); the stream is processed
 * in iterations of fixed-size batches (Section 3.1); a full window discards
 * its oldest value (Section 3.2).  Groups are spread over GPU workers by a
 * load balancer decided on the device from the batch's own key histogram
 * (the paper decides on the CPU and applies it one iteration late,
 * Section 3.1 and Section 4).
 *
 * Conventions for every call:
 *   - plain C types only; device pointers are HIP device (or managed)
 *     addresses; `stream` is a hipStream_t passed as void* (NULL = the
 *     default stream);
 *   - calls on one query are stream-ordered and must be issued on one
 *     stream (or ordered by the caller); a query is not thread-safe;
 *     distinct queries are independent;
 *   - no call throws; every call returns a CQ_* status code.
 *
 * Semantics taken where the paper is silent:
 *   - within a batch, arrival order is array order;
 *   - results are produced once per batch, for every group the batch
 *     touched, in ascending group id, with the value after that group's last
 *     tuple in the batch;
 *   - a window that is not yet full aggregates the values present:
 *     COUNT = min(window, tuples seen), AVG = (double)SUM / (double)COUNT,
 *     one IEEE-754 binary64 round-to-nearest division of exact integers;
 *   - SUM is exact in int64 (|SUM| <= window * 2^31 < 2^53).
 */
#ifndef CQ_H
#define CQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Aggregate selection bits for cq_create.  All three are always maintained;
 * the mask records what the caller asked for. */
#define CQ_SUM   1u
#define CQ_COUNT 2u
#define CQ_AVG   4u

/* Status codes. */
#define CQ_OK             0
#define CQ_ERR_INVALID   -1   /* bad argument; nothing was enqueued       */
#define CQ_ERR_OOM       -2   /* device memory short; nothing leaked      */
#define CQ_ERR_KEY_RANGE -3   /* the batch held a key outside [0, groups) */
#define CQ_ERR_HIP       -4   /* a HIP runtime call failed                */

/* Work assignment of the per-group phase (see cq_set_partition). */
#define CQ_PARTITION_BALANCED    0
#define CQ_PARTITION_STATIC      1
/* The paper's load-balancing techniques (Section 4), on the static
 * workers: see cq_set_partition. */
#define CQ_PARTITION_GETFIRST    2
#define CQ_PARTITION_CHECKALL    3
#define CQ_PARTITION_PROBCHECK   4
#define CQ_PARTITION_BESTBALANCE 5
#define CQ_PARTITION_SHIFT       6
#define CQ_PARTITION_SHIFTLOCAL  7

/* Largest batch accepted by cq_push_batch. */
#define CQ_MAX_BATCH (1ll << 30)
/* Largest window accepted by cq_create (keeps (double)SUM exact). */
#define CQ_MAX_WINDOW ((1 << 22) - 1)

typedef struct cq_query cq_query;

/*
 * cq_create -- a new query with `groups` group ids and a window of `window`
 * tuples per group (Section 3: group identifier, integer attribute, fixed
 * size window; Section 3.2: one window per group in device memory).
 *   groups     : 1 .. 2^31-1; keys must lie in [0, groups).
 *   window     : 1 .. CQ_MAX_WINDOW.
 *   aggregates : non-empty subset of CQ_SUM | CQ_COUNT | CQ_AVG.
 *   out        : receives the handle.
 * Allocates the window store (groups * window * 4 bytes) and the per-group
 * state on the current HIP device, zero-filled; the library owns them until
 * cq_destroy.  Returns CQ_OK, CQ_ERR_INVALID, CQ_ERR_OOM (nothing leaked,
 * *out = NULL) or CQ_ERR_HIP.
 */
int cq_create(int64_t groups, int32_t window, uint32_t aggregates, cq_query **out);

/*
 * cq_reserve -- kept for callers that size buffers up front: every working
 * buffer is sized by cq_create (batches run in fixed-size sub-batches), so
 * no later call allocates.  Returns CQ_OK or CQ_ERR_INVALID (q NULL or
 * max_batch outside 0 .. CQ_MAX_BATCH).
 */
int cq_reserve(cq_query *q, int64_t max_batch);

/*
 * cq_set_partition -- how groups are assigned to GPU workers in the
 * per-group phase (Section 4 load balancing; Section 5.1 initial
 * assignment).
 *   CQ_PARTITION_BALANCED (default): every batch, light groups are packed
 *     into workgroups by tuple count and every heavy group gets its own
 *     workgroup, decided on the device from the batch's histogram;
 *   CQ_PARTITION_STATIC: `workers` workers (0 = 1024), worker w owns the
 *     equal, consecutive group range [ceil(w*groups/workers),
 *     ceil((w+1)*groups/workers)) and processes every tuple of its groups
 *     -- the paper's initial assignment with balancing turned off
 *     (Section 5.1).  Needs workers <= 4096 and at most 2048 groups per
 *     worker;
 *   CQ_PARTITION_GETFIRST .. CQ_PARTITION_SHIFTLOCAL: the static workers,
 *     starting from the same ranges, with the group-to-worker mapping
 *     revised on the host after every batch by that technique of Section 4
 *     from the batch's tuples per worker, taking effect from the next batch
 *     (Section 3.1: one iteration of delay).  Groups move whole; no worker
 *     is given more than 2048 groups.  Each push then waits for its
 *     batch's histogram on the host (the GPU keeps working meanwhile), as
 *     the paper's CPU coordinator does.
 * Results are identical in every mode.  Takes effect at the next push and
 * restarts a technique's mapping from the initial ranges.  Returns CQ_OK
 * or CQ_ERR_INVALID.
 */
int cq_set_partition(cq_query *q, int32_t mode, int32_t workers);

/*
 * cq_set_key_mod -- on = 1: the query takes each key as (uint32_t)key mod
 * groups, so one input stream can feed queries with different group
 * counts (a key never falls outside the range); on = 0 (the default): keys
 * are used as given and a key outside [0, groups) rejects its batch.
 * Takes effect at the next push.  Returns CQ_OK or CQ_ERR_INVALID.
 */
int cq_set_key_mod(cq_query *q, int32_t on);

/*
 * cq_set_policy_params -- parameters of the Section 4 techniques: the
 * imbalance threshold in tuples (the paper's threadThreshold, default
 * 1000) and probCheck's pot (0 < pot <= 1, default 0.5; Section 5.1).
 * Returns CQ_OK or CQ_ERR_INVALID.
 */
int cq_set_policy_params(cq_query *q, int64_t threshold, double pot);

/*
 * cq_policy_stats -- after a push under a Section 4 technique: out[0] =
 * groups moved after the last batch, out[1] / out[2] = the largest /
 * smallest tuples per worker of that batch under the mapping it ran with,
 * out[3] = groups moved since the technique was selected.  Zeros in the
 * other modes.  Returns CQ_OK or CQ_ERR_INVALID.
 */
int cq_policy_stats(cq_query *q, int64_t *out);

/*
 * cq_policy_apply -- one balancing step of technique `policy` on the host,
 * without a query or a device (the step cq_push_batch runs after a batch
 * under that technique).  The mapping is given and returned as ordered
 * lists: worker w's groups are wlist[wstart[w] .. wstart[w+1]) (wstart has
 * workers+1 entries, wlist `groups`; every group exactly once).  counts[g]
 * are the batch's tuples of group g.  keys[0 .. n) are the batch's group
 * ids in arrival order (host array): probCheck reads the tuples of the most
 * loaded worker in that order (Figure alg3) and needs them, with counts
 * equal to their histogram; the other techniques ignore them (keys may be
 * NULL with n = 0).  *moves receives the number of groups moved.  Returns
 * CQ_OK or CQ_ERR_INVALID (bad arguments, mapping, or keys).
 */
int cq_policy_apply(int32_t policy, int32_t workers, int64_t groups, const int32_t *counts,
                    const int32_t *keys, int64_t n, int32_t *wstart, int32_t *wlist,
                    int64_t threshold, double pot, int32_t max_keys, int64_t *moves);

/*
 * cq_push_batch -- apply one batch of n tuples (Section 3.1: one iteration
 * over a batch; Section 3.2: each tuple enters its group's window, a full
 * window discarding its oldest value).
 *   keys, values : caller-owned device arrays of n int32 each (SoA); they
 *                  must stay valid and unchanged until the enqueued work has
 *                  completed; the library keeps no reference after that.
 *   n            : 0 .. CQ_MAX_BATCH; n = 0 is a valid batch touching nothing.
 *   stream       : hipStream_t (void*), NULL = default stream.
 * Enqueues the whole update on `stream` and returns without waiting for the
 * device; the only exception is a query under one of the Section 4
 * techniques (cq_set_partition), whose host step waits for the batch's
 * histogram.  Every working buffer was sized by cq_create, so the call
 * allocates nothing (cq_set_telemetry's records are allocated at the first
 * push after they are turned on).  Host-side errors
 * (q NULL, n out of range, NULL arrays with n > 0) return CQ_ERR_INVALID and
 * enqueue nothing.  A key outside [0, groups) is found on the device: the
 * whole batch is rejected, the windows are left unchanged, and the next
 * cq_results reports it.
 */
int cq_push_batch(cq_query *q, const int32_t *keys, const int32_t *values, int64_t n,
                  void *stream);

/*
 * cq_results -- write the results of the most recently pushed batch, one
 * entry per group the batch touched, in ascending group id.
 *   ids       : device int32[cap]  group id          (may be NULL)
 *   sums      : device int64[cap]  SUM of the window (may be NULL)
 *   counts    : device int32[cap]  COUNT             (may be NULL)
 *   avgs      : device double[cap] AVG               (may be NULL)
 *   n_touched : device int64[1]    number of entries written (required)
 * with cap >= min(groups, n of that batch).  Stream-ordered after the push;
 * returns CQ_OK without waiting for the device.  If that batch was rejected
 * for a bad key, *n_touched receives CQ_ERR_KEY_RANGE (negative) and the
 * arrays are not written.  Before any push, *n_touched = 0.  The next push
 * replaces what this call reads.
 */
int cq_results(cq_query *q, int32_t *ids, int64_t *sums, int32_t *counts, double *avgs,
               int64_t *n_touched, void *stream);

/*
 * cq_push_batch_results -- cq_push_batch followed by cq_results into the
 * given device buffers, with the same arguments and the same results; the
 * per-group phase writes the results itself, saving the separate emission
 * launch.  For callers that want every batch's results (the per-batch
 * output of Section 3.1 iterations).
 */
int cq_push_batch_results(cq_query *q, const int32_t *keys, const int32_t *values, int64_t n,
                          int32_t *ids, int64_t *sums, int32_t *counts, double *avgs,
                          int64_t *n_touched, void *stream);

/*
 * cq_push_batch_results_noalloc -- cq_push_batch_results for callers that
 * cannot allocate device memory while they run: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, same state change and same results; the call allocates
 * nothing.  Its working memory (histogram, plan, reordered tiles) is one
 * fixed area of CQ_NOALLOC_SCRATCH_BYTES per GPU, a file-scope device array
 * that each GPU the library runs on holds until the process ends; the
 * caller still passes the inputs and the result buffers.
 * Limits: n <= CQ_NOALLOC_MAX_BATCH tuples, a query of at most
 * CQ_NOALLOC_MAX_GROUPS groups in the balanced partition (no Section 4
 * technique); anything beyond returns CQ_ERR_INVALID with nothing enqueued.
 * Every call on one GPU shares that area: calls that overlap on one GPU
 * (any query, any stream, not ordered one after the other) race and give
 * undefined results.  Each call first clears what must start at zero, so a
 * sequence of ordered calls (also replays of a captured one) is exact.  A
 * bad key rejects the batch (*n_touched = CQ_ERR_KEY_RANGE, state
 * unchanged).  After this call cq_results, cq_status and cq_batch_plan
 * return CQ_ERR_INVALID until the query's next push through another entry
 * point.  Telemetry is not recorded.  Returns CQ_OK, CQ_ERR_INVALID or
 * CQ_ERR_HIP.
 */
#define CQ_NOALLOC_MAX_BATCH 262144       /* 2^18 tuples */
#define CQ_NOALLOC_MAX_GROUPS 16384
#define CQ_NOALLOC_SCRATCH_BYTES 3145728  /* 3 MiB */
int cq_push_batch_results_noalloc(cq_query *q, const int32_t *keys, const int32_t *values,
                                  int64_t n, int32_t *ids, int64_t *sums, int32_t *counts,
                                  double *avgs, int64_t *n_touched, void *stream);

/* Limits of cq_push_batch_tuples. */
#define CQ_TUPLE_MAX_WINDOW 1024
#define CQ_TUPLE_MAX_GROUPS 2097152  /* 2^21 */
#define CQ_TUPLE_MAX_PASSES 64

/*
 * cq_push_batch_tuples -- apply one batch exactly as cq_push_batch does and,
 * for every tuple, report its group's aggregate right after that tuple
 * entered the window: the paper recomputes the aggregate after each
 * insertion by scanning the whole window (Section 5.1), and its last
 * experiment scans it ten times (Section 5.2, further experiments).
 *   sums[i], counts[i], avgs[i] : device arrays of n entries (any may be
 *       NULL), in arrival order: SUM (int64) of the window of keys[i]'s
 *       group after tuple i, COUNT = min(W, values seen), AVG =
 *       (double)SUM / (double)COUNT;
 *   passes : 0 = the sums follow incrementally (new value minus evicted
 *       value); 1 .. CQ_TUPLE_MAX_PASSES = every tuple's window is summed
 *       from scratch that many times (the paper's 1 and 10).  The results
 *       are the same integers either way.
 * Needs the balanced partition, at most CQ_TUPLE_MAX_GROUPS groups and a
 * window of at most CQ_TUPLE_MAX_WINDOW.  The first call allocates 4 MiB + 4 bytes per
 * group of device memory for the query.  Stream-ordered like cq_push_batch;
 * a rejected batch (bad key) writes no per-tuple entry and cq_status
 * reports it.  cq_results afterwards gives the batch's per-group results.
 * Returns CQ_OK, CQ_ERR_INVALID, CQ_ERR_OOM or CQ_ERR_HIP.
 */
int cq_push_batch_tuples(cq_query *q, const int32_t *keys, const int32_t *values, int64_t n,
                         int32_t passes, int64_t *sums, int32_t *counts, double *avgs,
                         void *stream);

/*
 * cq_push_batches -- `count` consecutive batches of one stream in one call:
 * the same state and the same per-batch results as cq_push_batch_results
 * on each batch in order (Section 3.1's iteration over incoming batches).
 *   keys[i], values[i] : device int32[n[i]] of batch i (host array of
 *                        device pointers), 0 <= n[i] <= 2^20 (CQ_PIPE_MAX)
 *   ids[i], sums[i], counts[i], avgs[i], n_touched[i] : batch i's result
 *                        buffers as for cq_results (the four arrays of
 *                        pointers may be NULL, n_touched[i] may not)
 * With the balanced partition and at most 16384 groups, up to
 * CQ_CHAIN_BATCHES batches share one set of six launches (histogram, two
 * plan launches, reorder, survivors, apply); a longer call is cut into
 * ceil(count / CQ_CHAIN_BATCHES) sets of near-equal size.  Otherwise
 * consecutive batches use two sets of batch-local buffers, so batch i+1's
 * key histogram is computed by extra workgroups of batch i's per-group
 * launch: two launches per batch instead of three.  Stream-ordered on
 * `stream`; returns without waiting for the device.  A batch with a bad key
 * gets CQ_ERR_KEY_RANGE in *n_touched[i] and leaves the state unchanged;
 * the other batches proceed.  The input and result buffers must stay valid
 * until the work on `stream` completes.  Telemetry records describe the
 * last batch.  Returns CQ_OK, CQ_ERR_INVALID (nothing enqueued), CQ_ERR_OOM
 * or CQ_ERR_HIP.
 */
#define CQ_PIPE_MAX 1048576 /* 2^20 tuples per batch */
#define CQ_CHAIN_BATCHES 20 /* batches per set of launches of cq_push_batches */
int cq_push_batches(cq_query *q, int32_t count, const int32_t *const *keys,
                    const int32_t *const *values, const int64_t *n, int32_t *const *ids,
                    int64_t *const *sums, int32_t *const *counts, double *const *avgs,
                    int64_t *const *n_touched, void *stream);

/*
 * cq_status -- wait for the query's last stream and return the status of the
 * most recent batch: CQ_OK or CQ_ERR_KEY_RANGE (or CQ_ERR_HIP).
 */
int cq_status(cq_query *q);

/*
 * cq_destroy -- wait for the query's last stream, then free everything.
 * NULL is a no-op returning CQ_OK.
 */
int cq_destroy(cq_query *q);

/* Static description of a status code. */
const char *cq_strerror(int code);

/* ------------------- many queries over one stream --------------------- */

/* Number of groups of a query (CQ_OK or CQ_ERR_INVALID). */
int cq_query_groups(const cq_query *q, int64_t *groups);

typedef struct cq_multi cq_multi;

#define CQ_MULTI_MAX_LANES 16

/*
 * cq_multi_create -- a set of `count` queries that all take the same input
 * batches (give them cq_set_key_mod when their group counts differ).  The
 * queries are spread over `lanes` HIP streams of their own (0 = 8, at most
 * CQ_MULTI_MAX_LANES, default priority), forked from and joined back into
 * the caller's stream by events: queries on different lanes overlap on the
 * device, each query's batches stay in order.  The set does not own the
 * queries (destroy them after the set).  Returns CQ_OK, CQ_ERR_INVALID,
 * CQ_ERR_OOM or CQ_ERR_HIP.
 */
int cq_multi_create(cq_query *const *queries, int32_t count, int32_t lanes, cq_multi **out);

/*
 * cq_multi_push -- apply one batch (device keys, values; n tuples) to every
 * query of the set, stream-ordered on `stream` (NULL = default stream): work
 * enqueued on `stream` afterwards, e.g. cq_results of any query, sees every
 * query updated.  During a tuning window the call also waits for the batch
 * on the host.  Returns CQ_OK, CQ_ERR_INVALID or CQ_ERR_HIP (a bad key
 * rejects that query's batch as in cq_push_batch).
 */
int cq_multi_push(cq_multi *m, const int32_t *keys, const int32_t *values, int64_t n,
                  void *stream);

/*
 * cq_multi_tune -- open a tuning window over the next pushes: every query
 * runs each of its candidate partitions (balanced; static with 1024 and with
 * 4096 workers where a worker would own at most 2048 groups) for `reps`
 * consecutive batches (1..64), timed on its lane; at the end of the window
 * each query keeps its fastest candidate (median) and the queries are
 * re-spread over the lanes longest first onto the least loaded lane.
 * Results are identical under every candidate.  Returns CQ_OK,
 * CQ_ERR_INVALID or CQ_ERR_HIP.
 */
int cq_multi_tune(cq_multi *m, int32_t reps);

/*
 * cq_multi_plan -- per query (host arrays of count entries, any may be
 * NULL): chosen partition mode and workers (-1 before a tuning window has
 * ended), lane, and the chosen candidate's median time in milliseconds
 * (-1 before tuning).  Returns CQ_OK or CQ_ERR_INVALID.
 */
int cq_multi_plan(cq_multi *m, int32_t *modes, int32_t *workers, int32_t *lanes, float *ms);

/*
 * cq_multi_set_graph -- on = 1: outside tuning windows, each push copies the
 * batch into staging buffers of the set and replays the set's whole
 * per-batch launch sequence (every query, every lane, fork and join) as one
 * HIP graph, captured on the first push of each batch size; on = 0: eager
 * pushes again.  The queries must have telemetry off and no Section 4
 * technique; their results and state are the same either way, and
 * cq_push_batch on a query of the set keeps working in between.  A new
 * tuning window or a larger batch drops the captured graphs.  Returns
 * CQ_OK, CQ_ERR_INVALID or CQ_ERR_HIP.
 */
int cq_multi_set_graph(cq_multi *m, int32_t on);

/* Waits for the set's lanes and frees them (not the queries). */
int cq_multi_destroy(cq_multi *m);

/* ------------------------------ serving ------------------------------- */

/*
 * cq_query_footprint -- device bytes a query of `groups` groups and window
 * `window` allocates (window store, per-group state and its working
 * buffers; each allocation rounded up to 4 KiB), or -1 for invalid sizes.
 */
int64_t cq_query_footprint(int64_t groups, int32_t window);

typedef struct cq_server cq_server;

#define CQ_SERVER_MAX_LANES 16
#define CQ_SERVER_MAX_SLOTS 64

/*
 * cq_server_create -- a serving loop on the current device: many resident
 * queries whose batches arrive over time (Section 3.1 takes one batch per
 * iteration as the stream delivers it; Section 3.2 keeps every window in
 * GPU memory).
 *   memory_budget : device bytes the resident queries may hold (0 = 80% of
 *                   the free device memory now);
 *   lanes         : HIP streams, default priority (0 = 8, at most
 *                   CQ_SERVER_MAX_LANES).  Each query is pinned to one lane,
 *                   so its batches run in submission order, while batches
 *                   of queries on other lanes overlap with them on the GPU;
 *   slots         : requests in flight per lane (0 = 2, at most
 *                   CQ_SERVER_MAX_SLOTS).
 * A dispatcher thread starts waiting requests in arrival order as slots
 * free up (a request never passes an earlier one of its own query).
 * Returns CQ_OK, CQ_ERR_INVALID, CQ_ERR_OOM or CQ_ERR_HIP.
 */
int cq_server_create(int64_t memory_budget, int32_t lanes, int32_t slots, cq_server **out);

/*
 * cq_server_add_query -- admit a query (as cq_create) if its footprint fits
 * the budget still free; *qid receives its id.  Returns CQ_OK,
 * CQ_ERR_INVALID, CQ_ERR_OOM (does not fit, nothing allocated) or
 * CQ_ERR_HIP.  cq_server_remove_query waits for the query's requests, frees
 * it and returns its bytes to the budget.
 */
int cq_server_add_query(cq_server *srv, int64_t groups, int32_t window, uint32_t aggregates,
                        int32_t *qid);
int cq_server_remove_query(cq_server *srv, int32_t qid);

/*
 * cq_server_submit -- queue one batch of query qid: device arrays keys,
 * values (n tuples), and result arrays exactly as cq_push_batch_results
 * (ids/sums/counts/avgs of min(groups, n) entries, any may be NULL;
 * n_touched required; a rejected batch gets its status there).  Every
 * array must stay valid until the request completes.  *ticket receives the
 * request's number.  Returns at once: CQ_OK or CQ_ERR_INVALID.
 */
int cq_server_submit(cq_server *srv, int32_t qid, const int32_t *keys, const int32_t *values,
                     int64_t n, int32_t *ids, int64_t *sums, int32_t *counts, double *avgs,
                     int64_t *n_touched, int64_t *ticket);

/*
 * cq_server_wait -- block until request `ticket` has completed on the GPU
 * (its results are then in place) and return its launch status; a ticket
 * can be waited for once.  ticket = -1 waits for every request submitted so
 * far and forgets their tickets.
 */
int cq_server_wait(cq_server *srv, int64_t ticket);

/*
 * cq_server_stats -- over the requests completed since the previous call:
 * out[0] requests, out[1] p50 and out[2] p99 and out[3] max latency in
 * microseconds (host clock, submission to observed completion), out[4]
 * tuples, out[5] tuples per second over the span from the earliest
 * submission to the last completion; out[6] / out[7] device bytes held /
 * budget.  Then starts counting afresh.
 */
int cq_server_stats(cq_server *srv, double *out);

/* Waits for every request, frees every query, the lanes and the server. */
int cq_server_destroy(cq_server *srv);

/* ---------------- measurement (not needed for results) ---------------- */

/* Telemetry flags for cq_set_telemetry. */
#define CQ_TELEMETRY_KERNEL_TIMES 1 /* HIP events around every kernel launch */
#define CQ_TELEMETRY_PHASES       4 /* device clock at fixed points inside each
                                       kernel, per workgroup (cq_phase_trace) */
#define CQ_TELEMETRY_WORKERS      2 /* per-workgroup (hardware id, start, end,
                                       tuples) records of the per-group phase */

/* Launch kinds reported by cq_kernel_times, in this order. */
#define CQ_KERNEL_HIST      0 /* key histogram                        */
#define CQ_KERNEL_PASS      1 /* tile-local reorder by bucket (and,
                                 for up to 16384 groups, the plan)   */
#define CQ_KERNEL_UPDATE    2 /* per-group evict + insert + aggregate */
#define CQ_KERNEL_EMIT      3 /* separate result emission             */
#define CQ_KERNEL_OTHER     4 /* whole-batch checks and collection    */
#define CQ_KERNEL_PLAN      5 /* scans over groups + balancer plan    */
#define CQ_KERNEL_TUPLES    6 /* per-tuple results (cq_push_batch_tuples) */
#define CQ_KERNEL_PREP      7 /* several batches: survivors to their places */
#define CQ_KERNEL_APPLY     8 /* several batches: windows, results, rings */
#define CQ_KERNEL_KINDS     9

/*
 * cq_set_telemetry -- turn measurement on (flags) or off (0).  Imbalance
 * is what the paper's balancing corrects (Section 1; Section 3.1 detects it
 * from tuples per thread); these records make it measurable on the device.
 * Returns CQ_OK, CQ_ERR_INVALID or CQ_ERR_OOM.
 */
int cq_set_telemetry(cq_query *q, int32_t flags);

/*
 * cq_kernel_times -- wait for the query's last stream; for every kernel
 * kind k < nkinds, write the summed duration in milliseconds of its launches
 * since the previous call to ms[k] and their number to launches[k]
 * (host arrays); then start counting afresh.  Needs
 * CQ_TELEMETRY_KERNEL_TIMES.  Returns CQ_OK, CQ_ERR_INVALID or CQ_ERR_HIP.
 */
int cq_kernel_times(cq_query *q, double *ms, int64_t *launches, int32_t nkinds);

/*
 * cq_worker_trace -- wait for the query's last stream and copy the
 * per-workgroup records of the most recent batch's per-group phase into the
 * host array `rec` (cap records of 6 int64: raw HW_ID register, XCC id,
 * start tick, end tick, tuples handled, items handled; ticks of the
 * constant 100 MHz device clock).  *count receives the number of records
 * available.  Needs CQ_TELEMETRY_WORKERS.
 */
int cq_worker_trace(cq_query *q, int64_t *rec, int64_t cap, int64_t *count);

/*
 * cq_phase_trace -- wait for the query's last stream and copy the phase
 * clocks of the most recent sub-batch for one kernel `kind` into the host
 * array `out` (cap records of 8 int64 device-clock ticks, one record per
 * workgroup, 0 = not reached).  kind 0: histogram (slots 0-2) and, where
 * the plan is a launch of its own, the plan (slots 3-4); kind 1: reorder
 * pass (slots 0-4; with the plan inside the pass, slots 5-7 mark its
 * steps); kind 2: per-group update (slots 0-5); several batches per call
 * (cq_push_batches): kind 0 slots 3-7 the plan, kind 3 the survivor launch
 * (slots 0-5), kind 4 the apply launch (slots 0-7).  *count receives the
 * number of records available (4096).  Needs CQ_TELEMETRY_PHASES.  Returns
 * CQ_OK, CQ_ERR_INVALID or CQ_ERR_HIP.
 */
int cq_phase_trace(cq_query *q, int32_t kind, int64_t *out, int64_t cap, int64_t *count);

/*
 * cq_batch_plan -- wait for the query's last stream and copy the most
 * recent batch's partition summary into the host array `out` (9 int64):
 * light buckets, heavy groups, light tuples, touched groups (whole batch),
 * buckets (light + heavy, or static workers), touched groups of the last
 * sub-batch, status, reorder tiles of the last sub-batch, and the library's
 * sticky internal-consistency bits (0 unless a kernel found a plan breaking
 * its own size bounds and skipped work rather than overrun a buffer).
 */
int cq_batch_plan(cq_query *q, int64_t *out);

#ifdef __cplusplus
}
#endif
#endif
