// Internal interface between the C-ABI runtime (cq_runtime.cpp) and the HIP
// kernels (cq_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cq.h"

namespace cq {

// ---------------------------------------------------------------- sizes --
// A batch is processed in sub-batches of at most SUB tuples (windows after
// B1 then B2 equal windows after B1||B2, so this is exact); results are
// emitted once, after the last sub-batch.
constexpr int SUB = 1 << 20;
static_assert(SUB == CQ_PIPE_MAX, "pipelined batches are single sub-batches");

// Histogram: arrival tiles of HIST_THREADS threads, HIST_KPT keys per thread
// (loaded together); per-tile counters are
// LDS arrays indexed by key while groups <= HIST_DIRECT_MAX_G, otherwise an
// open-addressing LDS hash of HIST_HASH_SLOTS slots over HIST_HASH_TILE tuples.
constexpr int HIST_THREADS = 1024;
constexpr int HIST_KPT = 8;
constexpr int HIST_TILE = HIST_THREADS * HIST_KPT;
constexpr int HIST_DIRECT_MAX_G = 32768;
constexpr int HIST_HASH_TILE = 4096;   // 256 workgroups for a 2^20 sub-batch
static_assert(HIST_HASH_TILE % HIST_THREADS == 0, "whole keys per thread in a hashed tile");
constexpr int HIST_HASH_LOG = 13;
constexpr int HIST_HASH_SLOTS = 1 << HIST_HASH_LOG;
static_assert(HIST_HASH_SLOTS >= 2 * HIST_HASH_TILE, "hash load factor <= 1/2");

// Multi-block plan for G > HIST_DIRECT_MAX_G (scan over groups): PLAN_CHUNK
// groups per block of PLAN_THREADS.
constexpr int PLAN_THREADS = 256;
constexpr int PLAN_KPT = 10;   // 2560 groups a block: 410 blocks for 2^20 groups
constexpr int PLAN_CHUNK = PLAN_THREADS * PLAN_KPT;
constexpr int PLAN_FIELDS = 3;   // light tuples, heavy groups, touched groups

// Balanced assignment: a group with >= HEAVY_MIN tuples in a sub-batch is
// heavy and becomes a bucket of its own; light groups are packed, in id
// order, into buckets of about LIGHT_BUDGET tuples (fewer than LIGHT_BUDGET
// + HEAVY_MIN).
constexpr int HEAVY_MIN = 512;
constexpr int LIGHT_BUDGET = 512;
constexpr int LIGHT_CAP = LIGHT_BUDGET + HEAVY_MIN;
constexpr int LIGHT_BITS = 10;   // positions inside a light bucket
static_assert(LIGHT_CAP <= (1 << LIGHT_BITS), "light positions must fit the match bits");
constexpr int NB_MAX = SUB / LIGHT_BUDGET + SUB / HEAVY_MIN + 2;

// Multisplit pass: tiles of PASS_TILE tuples, PASS_WAVES waves, each wave a
// contiguous chunk of PASS_TILE / PASS_WAVES tuples in 64-lane rounds.
constexpr int PASS_TILE = 4096;
constexpr int PASS_WAVES = 8;
constexpr int PASS_THREADS = 64 * PASS_WAVES;
constexpr int PASS_ROUNDS = PASS_TILE / PASS_THREADS;
constexpr int PASS_TILES_MAX = SUB / PASS_TILE;
// Up to PASS_LOCAL_G groups the plan is computed inside the pass: every
// pass block reduces the whole histogram itself and keeps each group's
// bucket in LDS (16-bit), so no separate plan launch is needed.
constexpr int PASS_LOCAL_G = 16384;
constexpr int PL_PER = (PASS_LOCAL_G + PASS_THREADS - 1) / PASS_THREADS;
static_assert(PL_PER % 4 == 0, "int4 histogram loads");
static_assert(PASS_THREADS * PL_PER <= PASS_LOCAL_G, "in-block plan loads stay in the histogram");
// Counters the histogram array holds: at least PASS_LOCAL_G, so that the
// in-block plan's loads need no bounds test.
inline int64_t hist_entries(int64_t G) { return G > PASS_LOCAL_G ? G : PASS_LOCAL_G; }
static_assert(NB_MAX < 65536, "16-bit bucket ids");
__host__ __device__ constexpr bool plan_fused(int64_t G) { return G <= PASS_LOCAL_G; }
static_assert(PASS_TILE / PASS_WAVES < 65536, "per-wave counters are 16-bit");

// Per-group phase.
constexpr int UPD_THREADS = 256;
// Accelerator complex dies (each with its own L2) of the target device.
constexpr int XCDS = 8;
// Static assignment: one wave per worker, four workers per workgroup; a
// worker owns at most STATIC_KEYS_MAX groups.
constexpr int STATIC_WORKERS_PER_WG = 4;
constexpr int STATIC_KEYS_MAX = 2048;
constexpr int EMIT_THREADS = 256;

// Totals of the most recent (sub-)batch plan (device resident).
struct PlanTotals {
    int32_t n_light_buckets;
    int32_t n_heavy;
    int32_t light_tuples;   // tuples in light buckets
    int32_t n_touched;      // groups touched by the whole batch (final list)
    int32_t status;         // 0 or CQ_ERR_KEY_RANGE
    int32_t n_buckets;      // light + heavy (balanced) or workers (static)
    int32_t tiles;          // multisplit tiles of the last sub-batch
    int32_t sub_touched;    // groups touched by the last sub-batch
};

// Window store and per-group state.
struct State {
    int64_t G;
    int32_t W;
    int32_t *ring;   // G x W values; row g is group g's ring
    int32_t *pos;    // G: next ring slot (= tuples seen mod W)
    int32_t *cnt;    // G: values in the window (<= W)
    int64_t *sum;    // G: exact window sum
};

// Working buffers.
struct Scratch {
    // per group (G or G+1 entries)
    int32_t *k;         // histogram of the current sub-batch; zero between uses
    int32_t *lpre;      // G+1: exclusive prefix of tuples staged in light buckets
    int32_t *bucket;    // bucket of each touched group
    int32_t *pold;      // ring slot of each touched group before the sub-batch
    int32_t *tidx;      // output position of each touched group
    int32_t *stamp;     // batch sequence number that last touched the group
    int32_t *touched;   // touched group ids, ascending
    int32_t *ncnt;      // window count after this batch (emitted; the state may move on)
    // per bucket / heavy group
    int32_t *bstart;    // light bucket -> first group; [n_light] = G
    int32_t *hkey;      // heavy index -> group
    // multisplit output
    int2 *sdat;         // SUB staged (key, value), tile-major, bucket-sorted per tile
    int32_t *rowstart;  // [tile][n_buckets + 1] bucket starts inside each tile
    // control
    int32_t *partials;  // plan block partials
    int32_t *bad;       // batch sequence number of the last batch with a bad key
    int32_t *seqp;      // null, or (pushes captured into a graph) the device copy of
                        // the batch sequence number, advanced by the push itself
    int32_t *fault;     // sticky internal-consistency bits
    int32_t *hot;       // [2] most frequent groups of the last planned sub-batch
    PlanTotals *tot;
    // group-to-worker mapping of a Section 4 technique on the static
    // workers (null: the contiguous initial ranges)
    const int32_t *owner;   // G: worker of each group
    const int32_t *wstart;  // workers + 1: each worker's first list entry
    const int32_t *wlist;   // G: groups in worker-list order
    const int32_t *lidx;    // G: position of each group in its worker's list
    // keys reduced mod G (0: keys used as given): the multiplier of the
    // division-free remainder, floor((2^64 - 1) / G) + 1 (1 for G = 1)
    uint64_t kmod;
    // per-tuple results only (null otherwise)
    int32_t *sidx;      // SUB: arrival index of each staged tuple
    int32_t *pcnt;      // G: window count of each touched group before the sub-batch
    int64_t *trace;     // optional per-workgroup records (6 int64 each)
    int64_t *phase;     // optional phase clocks [kind][block][PHASE_SLOTS]
};

// Phase clocks (telemetry): kernels of kind PHASE_* record the device clock
// at fixed points, per workgroup, for the first PHASE_BLOCKS workgroups.
constexpr int PHASE_HIST_PLAN = 0;
constexpr int PHASE_PASS = 1;
constexpr int PHASE_UPDATE = 2;
constexpr int PHASE_SB_PREP = 3;   // several-batch survivor launch
constexpr int PHASE_SB_APPLY = 4;  // several-batch apply launch
constexpr int PHASE_KINDS = 5;
constexpr int PHASE_BLOCKS = 4096;
constexpr int PHASE_SLOTS = 8;

// Result destination of an emitting launch (all may be null).
struct Out {
    int32_t *ids;
    int64_t *sums;
    int32_t *counts;
    double *avgs;
    int64_t *n_touched;
};

// Several consecutive batches through one set of launches (cq_push_batches
// with at most PASS_LOCAL_G groups, balanced partition): up to SB_K batches
// of at most SUB tuples each share a histogram, a plan, a reorder, a
// survivor (prep) and an apply launch.  Each batch keeps its own balanced
// plan; the survivors of all batches -- a group's last min(k, W) tuples of
// each batch, which are the only ones any emitted window holds -- get
// consecutive places per group (batch by batch, arrival order), so that
// every batch's window sums are differences of prefix sums.
constexpr int SB_K = CQ_CHAIN_BATCHES;
// The several-batch path's buckets: a group with at least SB_HEAVY_MIN
// tuples of a batch is heavy, the others are packed into buckets of about
// SB_LIGHT_BUDGET tuples (fewer than SB_LIGHT_CAP).  Fewer, larger buckets
// than the single-batch path's: the reorder's per-wave counters then leave
// room for two workgroups per CU.
constexpr int SB_LIGHT_BUDGET = 1024;
constexpr int SB_HEAVY_MIN = 1024;
constexpr int SB_LIGHT_CAP = SB_LIGHT_BUDGET + SB_HEAVY_MIN;
constexpr int SB_NB_MAX = SUB / SB_LIGHT_BUDGET + SUB / SB_HEAVY_MIN + 2;
static_assert(SB_NB_MAX <= NB_MAX, "the bucket tables are sized for the single-batch bound");
// histogram blocks of the several-batch path (SBH_THREADS threads) count
// SBH_KPT keys per thread of one batch and store every group's count (16
// bits) of their tile; the plan sums a group's tiles
constexpr int SBH_THREADS = 512;
constexpr int SBH_KPT = 64;
constexpr int SBH_TILE = SBH_THREADS * SBH_KPT;
constexpr int SBH_TILES = (SUB + SBH_TILE - 1) / SBH_TILE;  // per batch at most
static_assert(SBH_TILE < 65536, "a tile's count of a group fits 16 bits");
static_assert(SBH_TILES < 256 && SB_NB_MAX < 65536, "a dropped-tile count and a bucket id share an int");
// plan: one group per thread in blocks of SBP_THREADS; per block of the first
// launch SBP_F field sums and two (count << 32 | group) words
constexpr int SBP_THREADS = 256;
constexpr int SBP_F = 2 * SB_K + 2;
constexpr int SBP_PART = SBP_F + 4;
// the plan's first launch: blocks of SBS_GROUPS groups
constexpr int SBS_GROUPS = 64;
constexpr int SBS_THREADS = SB_K * SBS_GROUPS / 2;
constexpr int SBS_BLOCKS_MAX = (PASS_LOCAL_G + SBS_GROUPS - 1) / SBS_GROUPS;
static_assert(SBS_BLOCKS_MAX % 64 == 0, "the plan's lanes stride over whole rows of blocks");
static_assert(SBP_THREADS % SBS_GROUPS == 0, "a plan block covers whole sums blocks");
static_assert(SBP_PART % 2 == 0, "the top-two words of a block's partials are 8-byte aligned");
// apply: a group whose survivors plus old window values read exceed
// APPLY_BUDGET is summed by a whole workgroup, every other one by one wave
constexpr int APPLY_BUDGET = 2048;
constexpr int APPLY_THREADS = 256;
// Workgroups of the reorder, survivor and apply launches, which loop over
// their items: as many as the device runs at once (256 CUs; two, three and
// four per CU fit their registers and LDS).
constexpr int SB_PREP_GRID = 768;
constexpr int SB_PASS_GRID = 512;
constexpr int SB_APPLY_GRID = 1024;

// Buffers of the several-batch path, one slice per batch where marked.
struct SbBufs {
    uint32_t *kt;       // [SB_K][SBH_TILES][(G + 1) / 2] per histogram tile, groups
                        // 2i and 2i + 1 in the low and high 16 bits of word i
    int32_t *kh;        // [G][SB_K] per-batch histograms, a group's counts together
    uint8_t *cut;       // [G][SB_K] a heavy group's leading histogram tiles holding
                        // none of its last W tuples of the batch
    int32_t *sbad;      // [SB_K] sequence number of the last call whose batch b had a bad key
    int32_t *bucket;    // [SB_K][G]
    int32_t *lpre;      // [SB_K][G + 1]
    int32_t *tidx;      // [SB_K][G]
    int32_t *bstart;    // [SB_K][NB_MAX + 1]
    int32_t *hkey;      // [SB_K][NB_MAX]
    int2 *sdat;         // [SB_K][SUB]
    int32_t *rowstart;  // [SB_K][PASS_TILES_MAX * (NB_MAX + 1)]
    PlanTotals *tot;    // [SB_K]
    int32_t *so;        // [SB_K][G] first place of batch b's survivors of group g
    int32_t *gsb;       // [G + 1] first place of group g's survivors
    int32_t *big;       // [G] the groups over APPLY_BUDGET, in group order
    int32_t *gbig;      // [G] 1 for those groups, else 0
    int32_t *xs;        // [SB_K * SUB] survivors' values, by group, batch, arrival
    int32_t *ntot;      // [2] groups over APPLY_BUDGET, survivors
    int64_t *tb;        // [SB_K][G] sum of a heavy item's survivors (batch, group)
    int32_t *part;      // [plan blocks][SBP_PART] plan fields summed per block, top two groups
    int32_t *fault;     // the query's fault bits
};

// The batches of one several-batch call (kernel argument).
struct SbBatches {
    const int32_t *keys[SB_K];
    const int32_t *values[SB_K];
    int64_t n[SB_K];
    int32_t htile0[SB_K + 1];   // histogram tiles before each batch
    int32_t ptile0[SB_K + 1];   // reorder tiles before each batch
    uint32_t vec;               // bit b: batch b's keys are 16-byte aligned
    int32_t K;
    Out out[SB_K];
};

// Batch b's slice of the several-batch buffers as a Scratch (with the
// query's shared pointers from `base`).
__host__ __device__ inline Scratch sb_set(const SbBufs &sb, const Scratch &base, int b,
                                          int64_t G) {
    Scratch s = base;
    s.k = nullptr;  // (the counters are interleaved by group: sb.kh[g * SB_K + b])
    s.bad = sb.sbad + b;
    s.bucket = sb.bucket + (int64_t)b * G;
    s.lpre = sb.lpre + (int64_t)b * (G + 1);
    s.tidx = sb.tidx + (int64_t)b * G;
    s.bstart = sb.bstart + (int64_t)b * (NB_MAX + 1);
    s.hkey = sb.hkey + (int64_t)b * NB_MAX;
    s.sdat = sb.sdat + (int64_t)b * SUB;
    s.rowstart = sb.rowstart + (int64_t)b * PASS_TILES_MAX * (NB_MAX + 1);
    s.tot = sb.tot + b;
    s.sidx = nullptr;
    s.pcnt = nullptr;
    s.trace = nullptr;
    return s;
}
// The launches of `in.K` batches, six in all (the plan is two; seq: the
// call's sequence number).
hipError_t launch_sb_hist(State st, Scratch base, SbBufs sb, const SbBatches &in, int32_t seq,
                          hipStream_t s);
hipError_t launch_sb_plan(State st, Scratch base, SbBufs sb, const SbBatches &in, int32_t seq,
                          hipStream_t s);
hipError_t launch_sb_pass(State st, Scratch base, SbBufs sb, const SbBatches &in, int32_t seq,
                          hipStream_t s);
hipError_t launch_sb_prep(State st, Scratch base, SbBufs sb, const SbBatches &in,
                          hipStream_t s);
hipError_t launch_sb_apply(State st, Scratch base, SbBufs sb, const SbBatches &in, int32_t seq,
                           hipStream_t s);

constexpr int32_t FAULT_LIGHT_SIZE = 1;
constexpr int32_t FAULT_BUCKETS = 2;
constexpr int32_t FAULT_STATIC_KEYS = 4;
constexpr int32_t FAULT_TUPLE_RUNS = 8;   // a bucket's runs disagree with its plan
constexpr int32_t FAULT_PASSES = 16;      // repeated window scans disagreed
constexpr int32_t FAULT_APPLY = 32;       // an apply range over its element budget

// Per-tuple results (the paper's aggregate after every insertion): one
// entry per tuple, in arrival order; any pointer may be null.  passes = 0:
// the window sum follows incrementally; passes >= 1: every tuple's window
// is summed from scratch that many times.
struct PtOut {
    int64_t *sums;
    int32_t *counts;
    double *avgs;
    int32_t passes;
};
constexpr int PT_WMAX = CQ_TUPLE_MAX_WINDOW;  // largest window of the per-tuple variant
constexpr int PT_CH = 1024;                   // ranks of a heavy group per work item
static_assert(PT_CH >= PT_WMAX, "only a heavy group's first item reaches back before rank W");

enum Mode { MODE_BALANCED = 0, MODE_STATIC = 1 };

// Launch sequence pieces (each enqueues on `s`, returns the launch status).
hipError_t launch_validate(const int32_t *keys, int64_t n, int64_t G, int32_t seq, Scratch sc,
                           hipStream_t s);
hipError_t launch_hist(const int32_t *keys, int64_t n, int64_t G, Scratch sc, int32_t seq,
                       hipStream_t s);
hipError_t launch_plan(State st, Scratch sc, int32_t seq, int mode, int32_t workers,
                       hipStream_t s);
hipError_t launch_pass(const int32_t *keys, const int32_t *values, int64_t n, State st,
                       Scratch sc, int32_t seq, int mode, int32_t workers, hipStream_t s);
// The next batch's histogram, computed by extra workgroups of an update
// launch (pipelined calls); blocks = 0 means none.
struct NextHist {
    const int32_t *keys;
    int64_t n;
    bool vec;
    int32_t blocks;
    int32_t seq;
    Scratch sc;
};
// Whether the next batch's histogram can ride along with an update launch.
bool can_fuse_hist(int64_t G, int mode);
hipError_t launch_update(State st, Scratch sc, int64_t n, int mode, int32_t workers, Out out,
                         hipStream_t s, const int32_t *next_keys = nullptr, int64_t next_n = 0,
                         Scratch next_sc = Scratch{}, int32_t next_seq = 0);
// Per-tuple results of the planned and reordered sub-batch (n tuples);
// reads the window store before the update launch changes it.
hipError_t launch_tuples(State st, Scratch sc, int64_t n, PtOut out, hipStream_t s);
hipError_t launch_collect_touched(int64_t G, int32_t seq, Scratch sc, hipStream_t s);
hipError_t launch_emit(State st, Scratch sc, int64_t cap, Out out, hipStream_t s);
hipError_t launch_reset_totals(Scratch sc, hipStream_t s);
// Advances the device copy of the batch sequence number by one.
hipError_t launch_bump_seq(Scratch sc, hipStream_t s);
// Sets the device copy of the batch sequence number.
hipError_t launch_set_seq(Scratch sc, int32_t v, hipStream_t s);
hipError_t launch_set_touched(int64_t *n_touched, int64_t v, hipStream_t s);
// Graph capture of pushes (multi-query sets): see cq_runtime.cpp.
bool query_capturable(const cq_query *q);
int query_set_graph(cq_query *q, bool on, hipStream_t s);
void query_replayed(cq_query *q, int64_t n, hipStream_t s);
void query_ran_on(cq_query *q, hipStream_t s);
// Working memory of the allocation-free push (cq_noalloc.hip): the scratch
// area's address on `device` (current), and the batch-local buffers carved
// out of it; launch_noalloc_clear zeroes the histogram and bad-key flag.
char *noalloc_base(int device);
Scratch noalloc_set(char *base);
hipError_t launch_noalloc_clear(const Scratch &sc, hipStream_t s);
// Workgroups of the per-group phase (one trace record each).
int64_t update_grid(int64_t n, int mode, int32_t workers);
// Histogram workgroups launched by launch_hist for a sub-batch of n.
int64_t hist_blocks(int64_t n, int64_t G);

}  // namespace cq
