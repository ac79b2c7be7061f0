/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of the continuous
 * sliding-window group-by aggregate of Koutsoumpakis, Koutsoumpakis and
 * Gounaris, "Skew Handling in Aggregate Streaming Queries on GPUs"
 * (ADMS 2013).  It exists only to check the GPU library against.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no source with the GPU library.
 *
 * What is computed (Section 3, problem statement; Section 3.2, GPU
 * operations; Section 5.1, experimental setting):
 *   - every tuple is (id, attr): a group identifier and an integer value;
 *   - every group keeps a fixed-size count window: its last W values;
 *     when the window is full the oldest value is discarded, and a per-group
 *     pointer (nextPos in the paper) marks the slot of the oldest value;
 *   - the aggregate of a group is recomputed from scratch over its window.
 *
 * Readings where the paper is silent:
 *   - tuples of a batch are applied in array order (arrival order);
 *   - results are emitted once per batch, for every group the batch touched,
 *     in ascending group id, with the value after the group's last tuple
 *     of the batch;
 *   - a partial window aggregates the values present: COUNT = min(W, seen);
 *   - SUM is int64, COUNT int32, AVG = (double)SUM / (double)COUNT;
 *   - a key outside [0, groups) rejects the whole batch, state unchanged.
 */
#ifndef CQ_ORACLE_H
#define CQ_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_query oracle_query;

/* 0 on success, -1 on invalid arguments, -2 when memory is short. */
int oracle_create(int64_t groups, int32_t window, oracle_query **out);
void oracle_destroy(oracle_query *q);

/* Apply one batch and write the per-touched-group results.  Output arrays
 * (any may be NULL) need room for min(groups, n) entries.  Returns 0, or -3
 * if a key is out of range (nothing changed, *n_touched = 0). */
int oracle_push(oracle_query *q, const int32_t *keys, const int32_t *values,
                int64_t n, int32_t *ids, int64_t *sums, int32_t *counts,
                double *avgs, int64_t *n_touched);

/* Same result, with groups split into `threads` contiguous ranges, one
 * thread each; every thread scans the whole batch and applies only its own
 * groups, so each group still sees its tuples in arrival order. */
int oracle_push_mt(oracle_query *q, const int32_t *keys, const int32_t *values,
                   int64_t n, int32_t *ids, int64_t *sums, int32_t *counts,
                   double *avgs, int64_t *n_touched, int threads);

/* The per-tuple form of Section 5.1: apply the batch tuple by tuple and,
 * after each insertion, write that group's window SUM (scanned from
 * scratch), COUNT and AVG at the tuple's own index (arrays of n entries,
 * any may be NULL).  The state afterwards is the same as oracle_push's.
 * Returns 0, or -3 if a key is out of range (nothing changed). */
int oracle_push_tuples(oracle_query *q, const int32_t *keys, const int32_t *values,
                       int64_t n, int64_t *sums, int32_t *counts, double *avgs);

/* Copy of one group's window in age order (oldest first); returns its
 * length (<= W).  For white-box tests of the ring. */
int32_t oracle_window(const oracle_query *q, int64_t group, int32_t *out);

#ifdef __cplusplus
}
#endif
#endif
