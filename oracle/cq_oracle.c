/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.  See cq_oracle.h for what it
 * computes and which readings of the paper it takes.
 *
 * Data layout mirrors the paper's description of the window store
 * (Section 3.2): one matrix holding a window of W slots for every group,
 * and a per-group pointer nextPos to the slot of the oldest value, which
 * moves on by one slot each time the oldest value is replaced.  The
 * aggregate is recomputed from scratch by scanning the whole window, as the
 * experimental setting does (Section 5.1), once per touched group at the
 * end of each batch (only that value is emitted).
 */
#include "cq_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

struct oracle_query {
    int64_t groups;     /* number of group ids: keys are 0 .. groups-1      */
    int32_t W;          /* window size in tuples                            */
    int32_t *windows;   /* groups x W values, row g = window of group g     */
    int32_t *nextPos;   /* per group: slot that the next value goes to;
                           once the window is full this is the oldest slot  */
    int32_t *filled;    /* per group: values currently in the window (<= W) */
    uint8_t *touched;   /* per group: touched by the current batch          */
};

int oracle_create(int64_t groups, int32_t window, oracle_query **out)
{
    if (!out || groups < 1 || groups > INT32_MAX || window < 1)
        return -1;
    *out = NULL;
    oracle_query *q = (oracle_query *)calloc(1, sizeof(*q));
    if (!q)
        return -2;
    q->groups = groups;
    q->W = window;
    q->windows = (int32_t *)calloc((size_t)groups * (size_t)window, sizeof(int32_t));
    q->nextPos = (int32_t *)calloc((size_t)groups, sizeof(int32_t));
    q->filled = (int32_t *)calloc((size_t)groups, sizeof(int32_t));
    q->touched = (uint8_t *)calloc((size_t)groups, 1);
    if (!q->windows || !q->nextPos || !q->filled || !q->touched) {
        oracle_destroy(q);
        return -2;
    }
    *out = q;
    return 0;
}

void oracle_destroy(oracle_query *q)
{
    if (!q)
        return;
    free(q->windows);
    free(q->nextPos);
    free(q->filled);
    free(q->touched);
    free(q);
}

/* Insert one value into group g's window: write it at nextPos (over the
 * oldest value when the window is full), then move nextPos on by one. */
static void window_insert(oracle_query *q, int64_t g, int32_t v)
{
    int32_t *win = q->windows + (size_t)g * (size_t)q->W;
    win[q->nextPos[g]] = v;
    q->nextPos[g] = (q->nextPos[g] + 1) % q->W;
    if (q->filled[g] < q->W)
        q->filled[g] += 1;
    q->touched[g] = 1;
}

/* The aggregate, from scratch: sum of every value in the window.  While the
 * window is not yet full its values sit in slots 0 .. filled-1. */
static int64_t window_sum(const oracle_query *q, int64_t g)
{
    const int32_t *win = q->windows + (size_t)g * (size_t)q->W;
    int64_t s = 0;
    for (int32_t j = 0; j < q->filled[g]; ++j)
        s += (int64_t)win[j];
    return s;
}

static int keys_valid(const oracle_query *q, const int32_t *keys, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (keys[i] < 0 || (int64_t)keys[i] >= q->groups)
            return 0;
    return 1;
}

/* Emit (id, SUM, COUNT, AVG) for touched groups in [g0, g1), ascending,
 * clearing their touched mark; returns how many were written. */
static int64_t emit_range(oracle_query *q, int64_t g0, int64_t g1, int32_t *ids,
                          int64_t *sums, int32_t *counts, double *avgs)
{
    int64_t m = 0;
    for (int64_t g = g0; g < g1; ++g) {
        if (!q->touched[g])
            continue;
        q->touched[g] = 0;
        int64_t s = window_sum(q, g);
        int32_t c = q->filled[g];
        if (ids)
            ids[m] = (int32_t)g;
        if (sums)
            sums[m] = s;
        if (counts)
            counts[m] = c;
        if (avgs)
            avgs[m] = (double)s / (double)c;
        ++m;
    }
    return m;
}

int oracle_push(oracle_query *q, const int32_t *keys, const int32_t *values,
                int64_t n, int32_t *ids, int64_t *sums, int32_t *counts,
                double *avgs, int64_t *n_touched)
{
    if (!q || n < 0 || (n > 0 && (!keys || !values)))
        return -1;
    if (n_touched)
        *n_touched = 0;
    if (!keys_valid(q, keys, n))
        return -3;
    for (int64_t i = 0; i < n; ++i)
        window_insert(q, keys[i], values[i]);
    int64_t m = emit_range(q, 0, q->groups, ids, sums, counts, avgs);
    if (n_touched)
        *n_touched = m;
    return 0;
}

int oracle_push_tuples(oracle_query *q, const int32_t *keys, const int32_t *values,
                       int64_t n, int64_t *sums, int32_t *counts, double *avgs)
{
    if (!q || n < 0 || (n > 0 && (!keys || !values)))
        return -1;
    if (!keys_valid(q, keys, n))
        return -3;
    /* Section 5.1: after every tuple enters its group's window, the whole
     * window is scanned and its sum computed from scratch */
    for (int64_t i = 0; i < n; ++i) {
        int64_t g = keys[i];
        window_insert(q, g, values[i]);
        int64_t ws = window_sum(q, g);
        int32_t wc = q->filled[g];
        if (sums)
            sums[i] = ws;
        if (counts)
            counts[i] = wc;
        if (avgs)
            avgs[i] = (double)ws / (double)wc;
    }
    /* the batch is over: clear the touched marks */
    emit_range(q, 0, q->groups, NULL, NULL, NULL, NULL);
    return 0;
}

typedef struct {
    oracle_query *q;
    const int32_t *keys, *values;
    int64_t n, g0, g1;
    int32_t *ids;
    int64_t *sums;
    int32_t *counts;
    double *avgs;
    int64_t m;
} mt_job;

static void *mt_worker(void *arg)
{
    mt_job *j = (mt_job *)arg;
    for (int64_t i = 0; i < j->n; ++i) {
        int64_t g = j->keys[i];
        if (g >= j->g0 && g < j->g1)
            window_insert(j->q, g, j->values[i]);
    }
    j->m = emit_range(j->q, j->g0, j->g1, j->ids, j->sums, j->counts, j->avgs);
    return NULL;
}

int oracle_push_mt(oracle_query *q, const int32_t *keys, const int32_t *values,
                   int64_t n, int32_t *ids, int64_t *sums, int32_t *counts,
                   double *avgs, int64_t *n_touched, int threads)
{
    if (!q || n < 0 || (n > 0 && (!keys || !values)) || threads < 1)
        return -1;
    if (n_touched)
        *n_touched = 0;
    if (!keys_valid(q, keys, n))
        return -3;
    if ((int64_t)threads > q->groups)
        threads = (int)q->groups;
    mt_job *jobs = (mt_job *)calloc((size_t)threads, sizeof(mt_job));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    int ok = jobs && tid;
    /* every thread emits into its own staging arrays, sized for the most
     * groups it can touch: min(size of its range, n) */
    for (int t = 0; ok && t < threads; ++t) {
        mt_job *j = &jobs[t];
        j->q = q; j->keys = keys; j->values = values; j->n = n;
        j->g0 = q->groups * t / threads;
        j->g1 = q->groups * (t + 1) / threads;
        int64_t cap = j->g1 - j->g0 < n ? j->g1 - j->g0 : n;
        size_t c = (size_t)(cap > 0 ? cap : 1);
        j->ids = (int32_t *)malloc(c * sizeof(int32_t));
        j->sums = (int64_t *)malloc(c * sizeof(int64_t));
        j->counts = (int32_t *)malloc(c * sizeof(int32_t));
        j->avgs = (double *)malloc(c * sizeof(double));
        ok = j->ids && j->sums && j->counts && j->avgs;
    }
    if (ok) {
        for (int t = 0; t < threads; ++t)
            pthread_create(&tid[t], NULL, mt_worker, &jobs[t]);
        for (int t = 0; t < threads; ++t)
            pthread_join(tid[t], NULL);
        /* ranges are ascending and disjoint: concatenating in thread order
         * keeps the output in ascending group id */
        int64_t m = 0;
        for (int t = 0; t < threads; ++t) {
            mt_job *j = &jobs[t];
            for (int64_t e = 0; e < j->m; ++e, ++m) {
                if (ids) ids[m] = j->ids[e];
                if (sums) sums[m] = j->sums[e];
                if (counts) counts[m] = j->counts[e];
                if (avgs) avgs[m] = j->avgs[e];
            }
        }
        if (n_touched)
            *n_touched = m;
    }
    for (int t = 0; jobs && t < threads; ++t) {
        free(jobs[t].ids); free(jobs[t].sums); free(jobs[t].counts); free(jobs[t].avgs);
    }
    free(jobs);
    free(tid);
    return ok ? 0 : -2;
}

int32_t oracle_window(const oracle_query *q, int64_t group, int32_t *out)
{
    if (!q || group < 0 || group >= q->groups)
        return -1;
    const int32_t *win = q->windows + (size_t)group * (size_t)q->W;
    int32_t f = q->filled[group];
    /* oldest value: slot 0 while filling, nextPos once full */
    int32_t start = (f < q->W) ? 0 : q->nextPos[group];
    for (int32_t j = 0; j < f; ++j)
        out[j] = win[(start + j) % q->W];
    return f;
}
