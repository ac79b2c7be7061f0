// Internal interface between the C-ABI runtime (cq_runtime.cpp) and the HIP
// kernels (cq_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cq {

// ---------------------------------------------------------------- tuning --
// Arrival tiles: the histogram and scatter kernels each take TILE
// consecutive tuples per 256-thread workgroup (ITEMS per thread).
constexpr int TILE = 2048;
constexpr int TILE_THREADS = 256;
constexpr int ITEMS = TILE / TILE_THREADS;
// A group with at least HEAVY_MIN tuples in a batch is heavy: it gets its
// own work item whose cost is bounded by the window, not by its tuples.
constexpr int HEAVY_MIN = 1024;
// Light groups are packed into buckets of about LIGHT_BUDGET tuples; a bucket
// holds fewer than LIGHT_BUDGET + HEAVY_MIN <= LCAP tuples.
constexpr int LIGHT_BUDGET = 1024;
constexpr int LCAP = 2048;
// Heavy run descriptors cached in LDS (beyond this they are re-read).
constexpr int DESC_CACHE = 2048;
// LDS counters indexed directly by key when groups <= DIRECT_MAX_G;
// otherwise an open-addressing LDS hash table with HASH_SLOTS slots.
constexpr int DIRECT_MAX_G = 12288;
constexpr int HASH_LOG = 12;
constexpr int HASH_SLOTS = 1 << HASH_LOG;
static_assert(HASH_SLOTS >= 2 * TILE, "hash load factor must stay <= 1/2");
static_assert(LIGHT_BUDGET + HEAVY_MIN <= LCAP, "light bucket bound");
// Plan (scan over groups): PLAN_THREADS threads x PLAN_KPT keys per block.
constexpr int PLAN_THREADS = 1024;
constexpr int PLAN_KPT = 16;
constexpr int PLAN_CHUNK = PLAN_THREADS * PLAN_KPT;
constexpr int PLAN_FIELDS = 5;
// Per-group phase workgroups.
constexpr int UPD_THREADS = 256;
constexpr int UPD_MAX_GRID = 4096;
constexpr int EMIT_THREADS = 256;

// Descriptor of one heavy run: the tuples of one heavy group that one
// arrival tile staged contiguously.  x = first staged slot; y = tile << 12 |
// (count - 1).
constexpr int RUN_COUNT_BITS = 12;
static_assert(TILE <= (1 << RUN_COUNT_BITS), "run count field");

// Totals of the most recent batch's plan (device resident).
struct PlanTotals {
    int32_t n_light_buckets;
    int32_t n_heavy;
    int32_t light_tuples;
    int32_t heavy_tuples;
    int32_t n_touched;
    int32_t n_desc;
    int32_t status;   // 0 or CQ_ERR_KEY_RANGE
    int32_t tiles;
};

// Bits of the device-side fault word (Scratch::fault): set when a kernel
// finds a plan that breaks one of its own size bounds and skips the work
// instead of overrunning a buffer.  Never set by a correct plan.
constexpr int32_t FAULT_LIGHT_SIZE = 1;
constexpr int32_t FAULT_HEAVY_CHUNK = 2;

// Window store and per-group state.
struct State {
    int64_t G;
    int32_t W;
    int32_t *ring;   // G x W values, row g is group g's ring
    int32_t *pos;    // G: next write slot of the ring (= tuples seen mod W)
    int32_t *cnt;    // G: values in the window (<= W)
    int64_t *sum;    // G: exact window sum
};

// Per-batch working buffers.
struct Scratch {
    int32_t *k;         // G   key histogram; zero between batches
    int32_t *lpre;      // G+1 exclusive prefix of light-group tuple counts
    int32_t *hcum;      // G+1 exclusive prefix of heavy flags (heavy index)
    int32_t *cursor;    // G   scatter cursor: next staged slot of the group
    int32_t *touched;   // G   touched group ids, ascending
    int32_t *hkey;      // heavy index -> group
    int32_t *hpre;      // heavy index -> first staged slot (relative); +1 end
    int32_t *hdb;       // heavy index -> first descriptor
    int32_t *hruns;     // heavy index -> descriptors written
    int2 *desc;         // heavy run descriptors
    int32_t *bkey;      // light bucket -> first group; [n_buckets] = G
    int2 *sdat;         // n staged (arrival index, value) pairs
    int32_t *partials;  // plan block partials (PLAN_FIELDS per block)
    int32_t *flag;      // [1] bad-key flag raised by the histogram
    int32_t *fault;     // [1] sticky FAULT_* bits (see above)
    PlanTotals *tot;    // plan totals
    int64_t *trace;     // optional per-workgroup records (6 int64 each)
};

// Launchers (each enqueues on `s` and returns the HIP launch status).
hipError_t launch_hist(const int32_t *keys, int64_t n, int64_t G, Scratch sc, hipStream_t s);
hipError_t launch_plan(int64_t G, int32_t tiles, Scratch sc, hipStream_t s);
hipError_t launch_scatter(const int32_t *keys, const int32_t *values, int64_t n, int64_t G,
                          Scratch sc, hipStream_t s);
hipError_t launch_update(State st, Scratch sc, int64_t n, int32_t tiles, int mode,
                         int32_t workers, hipStream_t s);
hipError_t launch_emit(State st, Scratch sc, int64_t cap, int32_t *ids, int64_t *sums,
                       int32_t *counts, double *avgs, int64_t *n_touched, hipStream_t s);
hipError_t launch_reset_totals(Scratch sc, hipStream_t s);
// Workgroups launched by launch_update (one trace record each).
int64_t update_grid(int64_t n, int mode, int32_t workers);

}  // namespace cq
