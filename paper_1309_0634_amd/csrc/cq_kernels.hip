// HIP kernels for gfx950 (CDNA4, wave64): one sub-batch (<= SUB tuples) of
// the continuous sliding-window group-by aggregate.
//
// Three launches per sub-batch (up to 16384 groups), in stream order:
//
//   k_hist_small  arrival tiles count keys in LDS (the previous sub-batch's
//                 two hottest keys in registers) and add their counts to
//                 the global histogram.
//   k_pass<true>  per arrival tile: the load balancer, then the reorder.
//                 Every workgroup reduces the whole histogram itself, so it
//                 knows each group's bucket without waiting on another
//                 (Section 4 moves groups between workers from per-worker
//                 tuple counts; here the exact per-group counts of this very
//                 batch decide, with no one-iteration delay): light groups
//                 are packed in id order into buckets of about LIGHT_BUDGET
//                 tuples, every group with >= HEAVY_MIN tuples becomes a
//                 bucket of its own, and each touched group's ring pointer
//                 moves on (Section 3.2: nextPos advances as values enter the
//                 window).  Then the tile's tuples are reordered by bucket,
//                 stably, in LDS and written back contiguously: the paper's
//                 two-pass linear reorder (Section 3.1), done per tile so
//                 that no tile waits on another.
//   k_update_*    the per-group phase: a bucket's tuples are read tile by
//                 tile (arrival order); every tuple among its group's last W
//                 goes to ring slot (pos + rank) mod W, and the group's sum
//                 gains (new value - value overwritten), i.e. the evicted
//                 value is subtracted (Section 3.2: a full window discards
//                 its oldest value).  Results are emitted in ascending group
//                 id.  In a pipelined call its first workgroups compute the
//                 next batch's histogram.
//
// More groups: a separate plan launch (k_plan_small, then k_pass<false>
// reads buckets from global memory), and beyond 32768 groups a hashed
// histogram (k_hist_hash) with a three-launch plan.
//
// Integer work bounded by memory traffic and latency: no MFMA.
#include <algorithm>

#include "cq.h"
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

// -------------------------------------------------------- plan (per key) --
// Fields scanned over groups: light tuples, heavy groups, touched groups.
__device__ __forceinline__ void key_fields(int32_t kg, int mode, int (&f)[PLAN_FIELDS]) {
    const bool heavy = mode == MODE_BALANCED && kg >= HEAVY_MIN;
    f[0] = (kg > 0 && !heavy) ? kg : 0;
    f[1] = heavy ? 1 : 0;
    f[2] = kg > 0 ? 1 : 0;
}

__device__ __forceinline__ int32_t static_worker(int64_t g, int64_t G, int32_t workers) {
    return (int32_t)((g * workers) / G);
}

// Plan of one touched group g with kg tuples, from the exclusive running
// field values x_ex (light tuples, heavy index, output position) and its
// current ring pointer po / count c: moves the ring pointer and count on (the
// update reads the old pointer from pold) and assigns the group's bucket.
__device__ __forceinline__ void plan_group(const State &st, const Scratch &sc, int64_t g,
                                           int32_t kg, const int (&x_ex)[PLAN_FIELDS],
                                           int32_t po, int32_t c, int32_t n_light, int32_t seq,
                                           int mode, int32_t workers) {
    const int32_t W = st.W;
    sc.stamp[g] = seq;
    sc.tidx[g] = x_ex[2];
    if ((uint32_t)x_ex[2] < (uint64_t)st.G) sc.touched[x_ex[2]] = (int32_t)g;
    sc.pold[g] = po;
    if (sc.pcnt) sc.pcnt[g] = c;
    st.pos[g] = (int32_t)(((uint32_t)po + (uint32_t)kg) % (uint32_t)W);
    const int32_t nc = (int32_t)min((int64_t)W, (int64_t)c + kg);
    st.cnt[g] = nc;
    sc.ncnt[g] = nc;  // the count emitted for this batch (the state may move on)
    if (mode == MODE_STATIC) {
        sc.bucket[g] = sc.owner ? sc.owner[g] : static_worker(g, st.G, workers);
    } else if (kg >= HEAVY_MIN) {
        sc.bucket[g] = n_light + x_ex[1];
        if ((uint32_t)x_ex[1] < (uint32_t)NB_MAX) sc.hkey[x_ex[1]] = (int32_t)g;
    } else {
        // light buckets: bucket m starts at the group whose staged range
        // [L, L + k) contains position m * LIGHT_BUDGET
        const int32_t L = x_ex[0];
        sc.bucket[g] = (L + kg - 1) / LIGHT_BUDGET;
        const int32_t m = (L + LIGHT_BUDGET - 1) / LIGHT_BUDGET;
        if ((int64_t)m * LIGHT_BUDGET <= (int64_t)L + kg - 1 && (uint32_t)m < (uint32_t)NB_MAX)
            sc.bstart[m] = (int32_t)g;
    }
}

// A plan block of the multi-block plan walks its groups in chunks; inside a
// chunk each wave owns PLAN_R rounds of 64 consecutive groups (lane =
// group), all loaded before use, so every load and store is coalesced.
// Prefixes come from DPP wave scans of two packed fields (light tuples;
// heavy flag | touched flag << 16), wave totals meet in LDS, and a running
// carry links the chunks.
constexpr int PLAN_R = 10;
// The packed field (heavy flag | touched flag << 16) is summed over at most
// one chunk of PLAN_THREADS * PLAN_R groups at a time (the running carry
// keeps the fields apart): the heavy half must stay below 2^16 and the
// whole sum below 2^31.
static_assert((int64_t)PLAN_THREADS * PLAN_R * 65537 < (1LL << 31),
              "packed per-chunk field sums fit an int, heavy count below 2^16");

// Top two (count << 32 | group) pairs of this thread's groups.
struct Top2 {
    unsigned long long a = 0, b = 0;
    __device__ void add(unsigned long long x) {
        if (x > a) { b = a; a = x; } else if (x > b) { b = x; }
    }
};

__device__ __forceinline__ void top2_wave(Top2 &t) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long xa = __shfl_xor(t.a, o, 64), xb = __shfl_xor(t.b, o, 64);
        t.add(xa);
        t.add(xb);
    }
}

__device__ void plan_publish(const State &st, const Scratch &sc, const int (&tot)[PLAN_FIELDS],
                             int32_t status, int mode, int32_t workers);

// Plans groups [gb, ge).  carry[q]: exclusive field values at gb on entry,
// at ge on exit (same in every thread).  `write`: emit the per-group plan
// and clear the histogram, unless per-tuple results follow (else only
// count).  Per-group plan writes happen
// only when `status` is 0.  `lds` holds 2 * waves ints.  Barriers inside.
__device__ void plan_range(const State &st, const Scratch &sc, int64_t gb, int64_t ge,
                           int (&carry)[PLAN_FIELDS], bool write, int32_t status,
                           int32_t n_light, int32_t seq, int mode, int32_t workers, int *lds) {
    const bool ok = status == 0;
    const int lane = lane_id(), wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t cb = gb; cb < ge; cb += (int64_t)nw * PLAN_R * 64) {
        // this lane's groups are g0 + 64 r; one base pointer per array and
        // constant offsets keep the address arithmetic out of the registers
        const int64_t g0 = cb + (int64_t)wv * PLAN_R * 64 + lane;
        const int32_t *kp = sc.k + g0;
        int32_t kv[PLAN_R], pv[PLAN_R], cv[PLAN_R];
#pragma unroll
        for (int r = 0; r < PLAN_R; ++r) {
            const bool in = g0 + 64 * r < ge;
            kv[r] = in ? kp[64 * r] : 0;
            pv[r] = (in && write && ok) ? st.pos[g0 + 64 * r] : 0;
            cv[r] = (in && write && ok) ? st.cnt[g0 + 64 * r] : 0;
        }
        int wa = 0, wb = 0;
#pragma unroll
        for (int r = 0; r < PLAN_R; ++r) {
            int x[PLAN_FIELDS];
            key_fields(kv[r], mode, x);
            wa += wave_total(wave_incl_add(x[0]));
            wb += wave_total(wave_incl_add(x[1] | (x[2] << 16)));
        }
        if (lane == 0) {
            lds[2 * wv] = wa;
            lds[2 * wv + 1] = wb;
        }
        __syncthreads();
        int before_a = 0, before_b = 0, all_a = 0, all_b = 0;
        for (int w = 0; w < nw; ++w) {
            const int xa = lds[2 * w], xb = lds[2 * w + 1];
            if (w < wv) { before_a += xa; before_b += xb; }
            all_a += xa;
            all_b += xb;
        }
        __syncthreads();
        if (write) {
            // the wave scans again (cheaper than holding every round's
            // prefixes in registers)
            int ra = carry[0] + before_a, rb = before_b;
            int32_t *kw = sc.k + g0, *lw = sc.lpre + g0;
#pragma unroll
            for (int r = 0; r < PLAN_R; ++r) {
                const int32_t kg = kv[r];
                int x[PLAN_FIELDS];
                key_fields(kg, mode, x);
                const int B = x[1] | (x[2] << 16);
                const int ia = wave_incl_add(x[0]), ib = wave_incl_add(B);
                const int ea = ra + ia - x[0], eb = rb + ib - B;
                ra += wave_total(ia);
                rb += wave_total(ib);
                // (the per-tuple step, after the plan, still reads the
                // counts of an accepted batch: the update clears them then)
                if (kg && (!sc.pcnt || !ok)) kw[64 * r] = 0;
                if (!ok || g0 + 64 * r >= ge) continue;
                int ex[PLAN_FIELDS] = {ea, carry[1] + (eb & 0xffff), carry[2] + (eb >> 16)};
                lw[64 * r] = ex[0];
                if (kg > 0)
                    plan_group(st, sc, g0 + 64 * r, kg, ex, pv[r], cv[r], n_light, seq, mode,
                               workers);
            }
        }
        carry[0] += all_a;
        carry[1] += all_b & 0xffff;
        carry[2] += all_b >> 16;
    }
}

// Block-wide top two over the threads' Top2 (result in thread 0); `nw`
// waves in the block.
__device__ void top2_block(Top2 &t, unsigned long long *lds, int nw) {
    const int wv = threadIdx.x >> 6;
    top2_wave(t);
    if (lane_id() == 0) {
        lds[2 * wv] = t.a;
        lds[2 * wv + 1] = t.b;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < nw; ++w) {
            t.add(lds[2 * w]);
            t.add(lds[2 * w + 1]);
        }
    __syncthreads();
}

// Totals of the plan; thread 0 only.
__device__ void plan_publish(const State &st, const Scratch &sc, const int (&tot)[PLAN_FIELDS],
                             int32_t status, int mode, int32_t workers) {
    const int32_t nl = mode == MODE_STATIC ? 0 : (tot[0] + LIGHT_BUDGET - 1) / LIGHT_BUDGET;
    PlanTotals t;
    t.n_light_buckets = nl;
    t.n_heavy = tot[1];
    t.light_tuples = tot[0];
    t.n_touched = tot[2];
    t.status = status;
    t.n_buckets = mode == MODE_STATIC ? workers : nl + tot[1];
    t.tiles = 0;
    t.sub_touched = tot[2];
    *sc.tot = t;
    if (!status) {
        if (mode != MODE_STATIC) sc.bstart[nl] = (int32_t)st.G;
        sc.lpre[st.G] = tot[0];
        if (t.n_buckets > NB_MAX) atomicOr(sc.fault, FAULT_BUCKETS);
    }
}

// ----------------------------------------------------- k_hist_plan (small G)
// Histogram tile `tile` (of `ntiles` counted into the same counters) of
// HIST_THREADS * KPT consecutive tuples of keys[0, n), one block of
// HIST_THREADS threads (every thread's KPT keys loaded together), LDS
// counters indexed by key (`cntr`, G of them), added to kout[g * kstride],
// or, with `dense`, every group's count stored there (16 bits, two groups a
// word); a bad key stores `seq` in *badout.
template <int KPT>
__device__ __forceinline__ void hist_small_tile(const int32_t *__restrict__ keys, int64_t n,
                                                bool vec, int32_t G, const Scratch &sc,
                                                int32_t seq, int tile, int ntiles,
                                                int32_t *kout, int kstride, int32_t *badout,
                                                int32_t *cntr) {
    static_assert(KPT % 4 == 0, "keys loaded four at a time");
    const int tid = threadIdx.x;
    phase_mark(sc, PHASE_HIST_PLAN, 0);
    // the previous sub-batch's two most frequent groups are counted in
    // registers: a Zipf-hot key would otherwise serialise LDS atomics
    const int32_t hot0 = sc.hot[0], hot1 = sc.hot[1];
    for (int g = tid; g < G; g += HIST_THREADS) cntr[g] = 0;
    const int64_t base = (int64_t)tile * HIST_THREADS * KPT;
    int32_t v[KPT];
#pragma unroll
    for (int j = 0; j < KPT / 4; ++j) {
        const int64_t i = base + 4 * ((int64_t)j * HIST_THREADS + tid);
        if (vec && i + 3 < n) {
            const int4 x = *reinterpret_cast<const int4 *>(keys + i);
            v[4 * j] = x.x; v[4 * j + 1] = x.y; v[4 * j + 2] = x.z; v[4 * j + 3] = x.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[4 * j + e] = (i + e < n) ? keys[i + e] : 0;
        }
    }
    if (sc.kmod) {
#pragma unroll
        for (int j = 0; j < KPT; ++j) v[j] = view_key(v[j], sc.kmod, G);
    }
    __syncthreads();
    int bad = 0, c0 = 0, c1 = 0;
#pragma unroll
    for (int j = 0; j < KPT / 4; ++j) {
        const int64_t i = base + 4 * ((int64_t)j * HIST_THREADS + tid);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (i + e >= n) continue;
            const int32_t key = v[4 * j + e];
            if (key < 0 || key >= G) bad = 1;
            else if (key == hot0) ++c0;
            else if (key == hot1) ++c1;
            else atomicAdd(&cntr[key], 1);
        }
    }
    c0 = wave_total(wave_incl_add(c0));
    c1 = wave_total(wave_incl_add(c1));
    if (lane_id() == 0) {
        if (c0) atomicAdd(&cntr[hot0], c0);
        if (c1) atomicAdd(&cntr[hot1], c1);
    }
    if (__syncthreads_or(bad)) {
        if (tid == 0) atomicExch(badout, seq);
    }
    phase_mark(sc, PHASE_HIST_PLAN, 1);
    // blocks start their flush at evenly spread groups, so that they do not
    // all hit the same counters at the same time
    const int off = (int)(((int64_t)tile * G / ntiles) & ~63);
    for (int i = tid; i < G; i += HIST_THREADS) {
        const int g = i + off < G ? i + off : i + off - G;
        const int32_t c = cntr[g];
        if (c) atomicAdd(&kout[(int64_t)g * kstride], c);
    }
    phase_mark(sc, PHASE_HIST_PLAN, 2);
}

// Histogram blocks over one sub-batch, tile = block.
__global__ __launch_bounds__(HIST_THREADS) void k_hist_small(const int32_t *__restrict__ keys,
                                                             int64_t n, bool vec, int32_t G,
                                                             Scratch sc, int32_t seq) {
    if (sc.seqp) seq = *sc.seqp;  // captured for replay: the argument would be stale
    extern __shared__ int32_t cntr[];
    hist_small_tile<HIST_KPT>(keys, n, vec, G, sc, seq, (int)blockIdx.x, (int)gridDim.x, sc.k, 1,
                              sc.bad, cntr);
}

// ------------------------------------------------- plan (G <= 32768) --
// One block per PS_THREADS consecutive groups, one group per thread.  Each
// block first reduces the fields over the whole histogram itself (at most
// 128 KB, from L2): that gives the totals and the exclusive field values at
// its first group with no inter-block communication.  Block 0 publishes the
// totals and keeps the two most frequent groups for the next histogram.
// The histogram is cleared by the per-group phase (every touched group
// belongs to exactly one bucket or worker), since other blocks of this
// launch still read it; a rejected batch is cleared here.
constexpr int PS_THREADS = 1024;
constexpr int PS_UNROLL = 16;

__global__ __launch_bounds__(PS_THREADS) void k_plan_small(State st, Scratch sc, int32_t seq,
                                                          int mode, int32_t workers) {
    if (sc.seqp) seq = *sc.seqp;  // captured for replay: the argument would be stale
    // The three fields (light tuples, heavy groups, touched groups) are
    // summed in separate ints: up to 32768 touched groups do not fit a
    // 16-bit half of a packed field.
    constexpr int NW = PS_THREADS / 64;
    __shared__ int red[2 * PLAN_FIELDS * NW];
    __shared__ unsigned long long red_top[2 * NW];
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int G = (int)st.G;
    const int gb = blockIdx.x * PS_THREADS;
    const int g = gb + tid;
    phase_mark(sc, PHASE_HIST_PLAN, 3);
    const int32_t status = *sc.bad == seq ? CQ_ERR_KEY_RANGE : 0;
    if (status) {
        if (g < G) sc.k[g] = 0;
        if (blockIdx.x == 0 && tid == 0) {
            const int none[PLAN_FIELDS] = {0, 0, 0};
            plan_publish(st, sc, none, status, mode, workers);
        }
        return;
    }
    // this thread's own group, loaded first
    const int32_t kg = g < G ? sc.k[g] : 0;
    const int32_t po = (g < G && kg > 0) ? st.pos[g] : 0;
    const int32_t c0 = (g < G && kg > 0) ? st.cnt[g] : 0;
    // per field: the sum over the groups before this block (b) and over all
    // groups (t) of this thread's share of the histogram
    int b[PLAN_FIELDS] = {0, 0, 0}, t[PLAN_FIELDS] = {0, 0, 0};
    const bool track = blockIdx.x == 0;
    Top2 top;
    for (int h0 = 0; h0 < G; h0 += PS_THREADS * PS_UNROLL) {
        int32_t kv[PS_UNROLL];
#pragma unroll
        for (int u = 0; u < PS_UNROLL; ++u) {
            const int h = h0 + u * PS_THREADS + tid;
            kv[u] = h < G ? sc.k[h] : 0;
        }
#pragma unroll
        for (int u = 0; u < PS_UNROLL; ++u) {
            const int h = h0 + u * PS_THREADS + tid;
            int x[PLAN_FIELDS];
            key_fields(kv[u], mode, x);
#pragma unroll
            for (int f = 0; f < PLAN_FIELDS; ++f) {
                t[f] += x[f];
                b[f] += h < gb ? x[f] : 0;
            }
            if (track && kv[u] > 0)
                top.add(((unsigned long long)(uint32_t)kv[u] << 32) | (uint32_t)h);
        }
    }
    // own group's exclusive position inside the block
    int x[PLAN_FIELDS], incl[PLAN_FIELDS];
    key_fields(kg, mode, x);
#pragma unroll
    for (int f = 0; f < PLAN_FIELDS; ++f) {
        incl[f] = wave_incl_add(x[f]);
        const int sb = wave_total(wave_incl_add(b[f]));
        const int stt = wave_total(wave_incl_add(t[f]));
        if (lane == 0) {
            red[(2 * wv) * PLAN_FIELDS + f] = sb;
            red[(2 * wv + 1) * PLAN_FIELDS + f] = stt;
        }
    }
    __shared__ int wtot[PLAN_FIELDS * NW];
    if (lane == 63) {
#pragma unroll
        for (int f = 0; f < PLAN_FIELDS; ++f) wtot[wv * PLAN_FIELDS + f] = incl[f];
    }
    __syncthreads();
    int ex[PLAN_FIELDS], tot[PLAN_FIELDS];
#pragma unroll
    for (int f = 0; f < PLAN_FIELDS; ++f) {
        int before_block = 0, all = 0, before_wave = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            before_block += red[(2 * w) * PLAN_FIELDS + f];
            all += red[(2 * w + 1) * PLAN_FIELDS + f];
            before_wave += w < wv ? wtot[w * PLAN_FIELDS + f] : 0;
        }
        ex[f] = before_block + before_wave + incl[f] - x[f];
        tot[f] = all;
    }
    const int32_t nl = mode == MODE_STATIC ? 0 : (tot[0] + LIGHT_BUDGET - 1) / LIGHT_BUDGET;
    if (blockIdx.x == 0 && tid == 0) plan_publish(st, sc, tot, status, mode, workers);
    if (g < G) {
        sc.lpre[g] = ex[0];
        if (kg > 0) plan_group(st, sc, g, kg, ex, po, c0, nl, seq, mode, workers);
    }
    if (track) {
        top2_block(top, red_top, NW);
        if (tid == 0) {
            sc.hot[0] = top.a ? (int32_t)(uint32_t)top.a : -1;
            sc.hot[1] = top.b ? (int32_t)(uint32_t)top.b : -1;
        }
    }
    phase_mark(sc, PHASE_HIST_PLAN, 4);
}

// ------------------------------------------------ histogram (large G) --
// HIST_HASH_TILE tuples per block; an LDS hash table aggregates equal keys,
// then one global atomic per distinct key.
__device__ __forceinline__ int hash_slot(int32_t *hk, int32_t key) {
    uint32_t h = ((uint32_t)key * 2654435761u) >> (32 - HIST_HASH_LOG);
    while (true) {
        const int32_t prev = atomicCAS(&hk[h], -1, key);
        if (prev == -1 || prev == key) return (int)h;
        h = (h + 1) & (HIST_HASH_SLOTS - 1);
    }
}

__global__ __launch_bounds__(HIST_THREADS) void k_hist_hash(const int32_t *__restrict__ keys,
                                                            int64_t n, int64_t G, int32_t seq,
                                                            Scratch sc) {
    if (sc.seqp) seq = *sc.seqp;  // captured for replay: the argument would be stale
    extern __shared__ int32_t lds[];
    int32_t *hk = lds, *hc = lds + HIST_HASH_SLOTS;
    const int tid = threadIdx.x;
    for (int s = tid; s < HIST_HASH_SLOTS; s += HIST_THREADS) {
        hk[s] = -1;
        hc[s] = 0;
    }
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * HIST_HASH_TILE;
    const int64_t b1 = min(n, b0 + HIST_HASH_TILE);
    // all of the thread's keys are loaded before any is hashed (indexes
    // clamped into the batch, n >= 1; positions past the tile are skipped)
    constexpr int KPT = HIST_HASH_TILE / HIST_THREADS;
    int32_t kv[KPT];
#pragma unroll
    for (int j = 0; j < KPT; ++j) kv[j] = keys[min(b0 + tid + j * HIST_THREADS, n - 1)];
    int bad = 0;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        if (b0 + tid + j * HIST_THREADS >= b1) continue;
        const int32_t key = view_key(kv[j], sc.kmod, G);
        if (key < 0 || (int64_t)key >= G) bad = 1;
        else atomicAdd(&hc[hash_slot(hk, key)], 1);
    }
    if (__syncthreads_or(bad)) {
        if (tid == 0) atomicExch(sc.bad, seq);
    }
    for (int s = tid; s < HIST_HASH_SLOTS; s += HIST_THREADS) {
        const int32_t key = hk[s];
        if (key >= 0) atomicAdd(&sc.k[key], hc[s]);
    }
}

// Plan over large G in three launches: block sums, a scan of the block
// sums, and the per-group writes.
__global__ __launch_bounds__(PLAN_THREADS) void k_plan_reduce(int64_t G, int mode, Scratch sc) {
    __shared__ int red[2 * (PLAN_THREADS / 64)];
    const int64_t gb = (int64_t)blockIdx.x * PLAN_CHUNK, ge = min(G, gb + PLAN_CHUNK);
    int tot[PLAN_FIELDS] = {0, 0, 0};
    State none{};
    plan_range(none, sc, gb, ge, tot, false, 0, 0, 0, mode, 1, red);
    if (threadIdx.x == 0)
        for (int q = 0; q < PLAN_FIELDS; ++q) sc.partials[blockIdx.x * PLAN_FIELDS + q] = tot[q];
}

__global__ __launch_bounds__(PLAN_THREADS) void k_plan_scan(int32_t nblk, State st, Scratch sc,
                                                            int32_t seq, int mode,
                                                            int32_t workers) {
    if (sc.seqp) seq = *sc.seqp;  // captured for replay: the argument would be stale
    __shared__ int red[PLAN_FIELDS * (PLAN_THREADS / 64)];
    const int per = (nblk + PLAN_THREADS - 1) / PLAN_THREADS;
    const int b0 = min(nblk, (int)threadIdx.x * per), b1 = min(nblk, b0 + per);
    int f[PLAN_FIELDS] = {0, 0, 0}, tot[PLAN_FIELDS];
    for (int b = b0; b < b1; ++b)
        for (int q = 0; q < PLAN_FIELDS; ++q) f[q] += sc.partials[b * PLAN_FIELDS + q];
    block_excl_scan<PLAN_FIELDS>(f, tot, red);
    for (int b = b0; b < b1; ++b)
        for (int q = 0; q < PLAN_FIELDS; ++q) {
            const int x = sc.partials[b * PLAN_FIELDS + q];
            sc.partials[b * PLAN_FIELDS + q] = f[q];
            f[q] += x;
        }
    if (threadIdx.x == 0) {
        const int32_t status = *sc.bad == seq ? CQ_ERR_KEY_RANGE : 0;
        plan_publish(st, sc, tot, status, mode, workers);
    }
}

// Per-group writes of the multi-block plan.  IN_BLOCK: every block sums the
// blocks' partials itself (those before it give its carry, all of them the
// totals, which block 0 publishes), so no scan launch runs between the two;
// the partials are read by every block, so this is kept to grids of at most
// PLAN_SCAN_IN_BLOCK_MAX blocks.  Otherwise k_plan_scan left each block's
// carry in its partials and the totals in `tot`.
constexpr int PLAN_SCAN_IN_BLOCK_MAX = 4 * PLAN_THREADS;  // blocks (2,621,440 groups)

template <bool IN_BLOCK>
__global__ __launch_bounds__(PLAN_THREADS) void k_plan_down(State st, Scratch sc, int32_t seq,
                                                            int mode, int32_t workers,
                                                            int32_t nblk) {
    if (sc.seqp) seq = *sc.seqp;  // captured for replay: the argument would be stale
    __shared__ int red[2 * PLAN_FIELDS * (PLAN_THREADS / 64)];
    const int64_t G = st.G;
    const int me = blockIdx.x, tid = threadIdx.x;
    const int64_t gb = (int64_t)me * PLAN_CHUNK, ge = min(G, gb + PLAN_CHUNK);
    int carry[PLAN_FIELDS];
    int32_t status, nl;
    if (IN_BLOCK) {
        // every partial this thread sums is loaded before any is added
        // (block indexes clamped into [0, nblk); the extra ones are skipped)
        constexpr int BPT = PLAN_SCAN_IN_BLOCK_MAX / PLAN_THREADS;
        int x[BPT][PLAN_FIELDS];
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int b = min(tid + j * PLAN_THREADS, nblk - 1);
#pragma unroll
            for (int q = 0; q < PLAN_FIELDS; ++q) x[j][q] = sc.partials[b * PLAN_FIELDS + q];
        }
        const int32_t bad = *sc.bad;
        int v[2 * PLAN_FIELDS] = {0, 0, 0, 0, 0, 0}, tot[2 * PLAN_FIELDS];
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int b = tid + j * PLAN_THREADS;
            if (b >= nblk) continue;
#pragma unroll
            for (int q = 0; q < PLAN_FIELDS; ++q) {
                v[q] += b < me ? x[j][q] : 0;  // blocks before this one
                v[PLAN_FIELDS + q] += x[j][q];  // all blocks
            }
        }
        block_excl_scan<2 * PLAN_FIELDS>(v, tot, red);  // (only the totals are used)
        const int all[PLAN_FIELDS] = {tot[PLAN_FIELDS], tot[PLAN_FIELDS + 1],
                                      tot[PLAN_FIELDS + 2]};
#pragma unroll
        for (int q = 0; q < PLAN_FIELDS; ++q) carry[q] = tot[q];
        status = bad == seq ? CQ_ERR_KEY_RANGE : 0;
        nl = mode == MODE_STATIC ? 0 : (all[0] + LIGHT_BUDGET - 1) / LIGHT_BUDGET;
        if (me == 0 && tid == 0) plan_publish(st, sc, all, status, mode, workers);
    } else {
#pragma unroll
        for (int q = 0; q < PLAN_FIELDS; ++q) carry[q] = sc.partials[me * PLAN_FIELDS + q];
        const PlanTotals t = *sc.tot;
        status = t.status;
        nl = t.n_light_buckets;
    }
    plan_range(st, sc, gb, ge, carry, true, status, nl, seq, mode, workers, red);
}

// Whole-batch key check (used when a batch spans several sub-batches, so
// that a bad key anywhere rejects the batch before any state changes).
__global__ void k_validate(const int32_t *__restrict__ keys, int64_t n, int64_t G, int32_t seq,
                           Scratch sc) {
    if (sc.seqp) seq = *sc.seqp;  // captured for replay: the argument would be stale
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t key = view_key(keys[i], sc.kmod, G);
        if (key < 0 || (int64_t)key >= G) bad = 1;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicExch(sc.bad, seq);
}

// --------------------------------------------------------------- k_pass --
// One arrival tile of PASS_TILE tuples per workgroup.  Wave w owns tuples
// [w*512, (w+1)*512) of the tile, visited in 64-lane rounds; every tuple
// learns its rank among the wave's earlier tuples of the same bucket from
// ballots over the bucket id bits (lanes of one bucket find each other)
// plus a per-wave counter.  Waves then combine into tile-wide bucket
// offsets, the tile is reordered in LDS and written back contiguously, and
// the tile's bucket starts are recorded.  Tiles never wait on each other.

// In-block plan of the fused pass (G <= PASS_LOCAL_G).  Every block reduces
// the whole histogram itself (thread t scans a contiguous run of groups),
// so each knows the bucket of every group without waiting on any other
// block: gbk[g] gets the bucket of each touched group (gcnt holds the
// counts meanwhile).  Block b writes the per-group plan of the contiguous
// groups [b*G/grid, (b+1)*G/grid); block 0 publishes the totals and keeps
// the two most frequent groups for the next histogram.  Returns the bucket
// count, or -1 for a rejected batch (whose histogram is cleared here: no
// block reads it then).  Barriers inside; call uniformly.
// Groups whose plan one pass workgroup writes per step of its in-block plan.
constexpr int OWN_CAP = 1024;
// The in-block plan sums the packed field (heavy flag | touched flag << 16)
// over all groups of the batch: at most PASS_LOCAL_G of each.
static_assert((int64_t)PASS_LOCAL_G * 65537 < (1LL << 31),
              "packed whole-histogram field sums fit an int, heavy count below 2^16");

// `load_tile` issues the tile's own loads.  It runs after the loads the plan
// waits on (the bad-key flag, the histogram, the owned groups' state), so the
// tile's tuples arrive while the plan is computed: loads complete in order.
template <typename F>
__device__ int pass_local_plan(const State &st, const Scratch &sc, int32_t seq, int mode,
                               int32_t workers, uint16_t *gbk, int32_t *gcnt, int4 *oex,
                               int *red, unsigned long long *red_top, int &own_n,
                               int32_t &po0, int32_t &c00, int32_t &nl_out, F &&load_tile) {
    // launched with PASS_THREADS threads (a constant: the block size would
    // otherwise be read from memory first)
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6, nw = PASS_WAVES;
    const int G = (int)st.G;
    const int D = gridDim.x, me = blockIdx.x;
    const bool bad = *sc.bad == seq;
    // this thread's groups [g0, g0 + R), R a multiple of 4 (int4 loads)
    const int R = ((G + PASS_THREADS - 1) / PASS_THREADS + 3) & ~3;
    const int g0 = tid * R;
    // exclusive fields at each run's start, beside the owned groups' fields
    int2 *runpre = reinterpret_cast<int2 *>(oex + OWN_CAP);
    // The histogram holds at least PASS_LOCAL_G >= PASS_THREADS * PL_PER
    // counters, so every load below is in bounds and is issued
    // unconditionally: a load under a divergent branch would be waited on
    // where the branch joins, one round trip after another.  Counts outside
    // the thread's run or past G are masked to zero.
    int32_t kv[PL_PER];
#pragma unroll
    for (int q = 0; q < PL_PER / 4; ++q) {
        const int g = g0 + 4 * q;
        const int4 x = *reinterpret_cast<const int4 *>(sc.k + g);
        const bool in = 4 * q < R;
        kv[4 * q] = in && g < G ? x.x : 0;
        kv[4 * q + 1] = in && g + 1 < G ? x.y : 0;
        kv[4 * q + 2] = in && g + 2 < G ? x.z : 0;
        kv[4 * q + 3] = in && g + 3 < G ? x.w : 0;
    }
    // this block writes the plan of groups [lo, hi), one group per thread
    // (in passes of OWN_CAP for a small grid); their state is loaded now
    const int lo = (int)((int64_t)me * G / D), hi = (int)((int64_t)(me + 1) * G / D);
    // (clamped into [0, G) and loaded unconditionally; read only by the
    // thread that owns group lo + tid < hi)
    const int gs = min(lo + tid, G - 1);
    po0 = st.pos[gs];
    c00 = st.cnt[gs];
    load_tile();
    if (bad) {
        for (int g = me * PASS_THREADS + tid; g < G; g += D * PASS_THREADS) sc.k[g] = 0;
        if (me == 0 && tid == 0) {
            const int none[PLAN_FIELDS] = {0, 0, 0};
            plan_publish(st, sc, none, CQ_ERR_KEY_RANGE, mode, workers);
        }
        return -1;
    }
    int sA = 0, sB = 0;
    const bool track = me == 0;
    Top2 top;
#pragma unroll
    for (int q = 0; q < PL_PER / 4; ++q) {
        if (4 * q >= R) break;  // (R is the same in every thread: a uniform branch)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * q + e;
            int x[PLAN_FIELDS];
            key_fields(kv[j], mode, x);
            sA += x[0];
            sB += x[1] | (x[2] << 16);
            if (track && kv[j] > 0)
                top.add(((unsigned long long)(uint32_t)kv[j] << 32) | (uint32_t)(g0 + j));
        }
    }
    // the run's counts into LDS (zeros past G included): the bucket loop
    // below reads them back there rather than keeping every count live
#pragma unroll
    for (int q = 0; q < PL_PER / 4; ++q)
        if (4 * q < R)
            *reinterpret_cast<int4 *>(gcnt + g0 + 4 * q) =
                make_int4(kv[4 * q], kv[4 * q + 1], kv[4 * q + 2], kv[4 * q + 3]);
    phase_mark(sc, PHASE_PASS, 5);
    const int iA = wave_incl_add(sA), iB = wave_incl_add(sB);
    if (lane == 63) {
        red[2 * wv] = iA;
        red[2 * wv + 1] = iB;
    }
    __syncthreads();
    phase_mark(sc, PHASE_PASS, 6);
    int bA = 0, bB = 0, TA = 0, TB = 0;
    for (int w = 0; w < nw; ++w) {
        const int xa = red[2 * w], xb = red[2 * w + 1];
        if (w < wv) {
            bA += xa;
            bB += xb;
        }
        TA += xa;
        TB += xb;
    }
    const int tot[PLAN_FIELDS] = {TA, TB & 0xffff, TB >> 16};
    const int32_t nl = mode == MODE_STATIC ? 0 : (TA + LIGHT_BUDGET - 1) / LIGHT_BUDGET;
    const int NB = mode == MODE_STATIC ? workers : nl + tot[1];
    if (me == 0 && tid == 0) plan_publish(st, sc, tot, 0, mode, workers);
    // Bucket of every group of the run.  This loop runs over all G groups in
    // every block, so it is kept free of branches: the mode is tested once,
    // heavy or light is a select, and the owned groups' fields are left to
    // the loop after it.  Untouched groups get an id too; it is never read.
    const int gend = min(G, g0 + R);
    nl_out = nl;
    const int eA0 = bA + iA - sA, eB0 = bB + iB - sB;  // exclusive fields at g0
    if (mode == MODE_STATIC && sc.owner) {  // a Section 4 mapping: buckets are workers
        for (int g = tid; g < G; g += PASS_THREADS) gbk[g] = (uint16_t)sc.owner[g];
    } else {
        int a = eA0, h = eB0 & 0xffff;  // light tuples and heavy groups before g
        // (gbk holds PASS_LOCAL_G ids, so the last int4 of a run past G is
        // stored whole)
        for (int g4 = g0; g4 < gend; g4 += 4) {
            const int4 c = *reinterpret_cast<const int4 *>(gcnt + g4);
            const int ks[4] = {c.x, c.y, c.z, c.w};
            uint32_t bo[4];
            if (mode == MODE_STATIC) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    bo[e] = ((uint32_t)(g4 + e) * (uint32_t)workers) / (uint32_t)G;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const bool heavy = ks[e] >= HEAVY_MIN;
                    const uint32_t light = (uint32_t)max(0, a + ks[e] - 1) / LIGHT_BUDGET;
                    bo[e] = heavy ? (uint32_t)(nl + h) : light;
                    a += heavy ? 0 : ks[e];
                    h += heavy ? 1 : 0;
                }
            }
            *reinterpret_cast<uint2 *>(gbk + g4) =
                make_uint2(bo[0] | (bo[1] << 16), bo[2] | (bo[3] << 16));
        }
    }
    // The exclusive fields and count of the groups this block owns, handed
    // through LDS to the threads that write their plan: consecutive groups
    // by consecutive lanes, so the plan's stores are coalesced.  Each owned
    // group's fields are rebuilt by one thread from the fields at the start
    // of the run that holds it (left in LDS by that run's thread) and the
    // counts before it in the run; the groups go round the waves, so that no
    // wave holds the block back at the next barrier.  With at most OWN_CAP
    // owned groups (every batch of 16 tiles or more) the writes happen
    // later, in the pass, after a barrier it needs anyway
    // (pass_owned_writes); a smaller grid takes OWN_CAP owned groups at a
    // time and writes them here.
    runpre[tid] = make_int2(eA0, eB0);
    __syncthreads();
    own_n = hi - lo <= OWN_CAP ? hi - lo : 0;
    const int spread = (tid & 63) * PASS_WAVES + (tid >> 6);  // lane-major over the waves
    int base = lo;
    do {
        const int top_g = min(hi, base + OWN_CAP);
        const bool first = base == lo;
        for (int i = spread; i < top_g - base; i += PASS_THREADS) {
            const int g = base + i;
            const int t = g / R, r0 = t * R;  // g's run and its first group
            const int2 p = runpre[t];
            int eA = p.x, eB = p.y;
#pragma unroll
            for (int q = 0; q < PL_PER / 4; ++q) {
                if (r0 + 4 * q >= g) break;
                const int4 c = *reinterpret_cast<const int4 *>(gcnt + r0 + 4 * q);
                const int ks[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = r0 + 4 * q + e < g ? ks[e] : 0;
                    const bool heavy = mode != MODE_STATIC && k >= HEAVY_MIN;
                    eA += heavy ? 0 : k;
                    eB += (heavy ? 1 : 0) + (k > 0 ? 1 << 16 : 0);
                }
            }
            oex[i] = make_int4(eA, eB, gcnt[g], 0);
        }
        if (own_n == 0 && top_g > base) {
            __syncthreads();
            for (int i = tid; i < top_g - base; i += PASS_THREADS) {
                const int g = base + i;
                const int4 e = oex[i];
                const int ex[PLAN_FIELDS] = {e.x, e.y & 0xffff, e.y >> 16};
                sc.lpre[g] = ex[0];
                if (e.z > 0) {
                    const bool pre = first && i == tid;
                    plan_group(st, sc, g, e.z, ex, pre ? po0 : st.pos[g], pre ? c00 : st.cnt[g],
                               nl, seq, mode, workers);
                }
            }
            __syncthreads();
        }
    } while ((base += OWN_CAP) < hi && own_n == 0);
    phase_mark(sc, PHASE_PASS, 7);
    if (track) {
        top2_block(top, red_top, PASS_WAVES);
        if (tid == 0) {
            sc.hot[0] = top.a ? (int32_t)(uint32_t)top.a : -1;
            sc.hot[1] = top.b ? (int32_t)(uint32_t)top.b : -1;
        }
    }
    __syncthreads();
    return NB;
}

// bytes of one wave's leader table in the multisplit: every bucket id has an
// entry (at most NB_MAX - 2 buckets: a static partition's workers, or about
// SUB / LIGHT_BUDGET + 1 balanced ones)
constexpr int LEAD = 2 * PASS_LOCAL_G / PASS_WAVES;
static_assert(LEAD >= NB_MAX - 2, "a leader entry for every bucket");
constexpr int P_WC = 0;                                            // u16[PASS_WAVES][NB_MAX]
static_assert(NB_MAX % 2 == 0, "per-wave counter rows are cleared as 32-bit pairs");
constexpr int P_STAGE = (P_WC + 2 * PASS_WAVES * NB_MAX + 15) & ~15;  // int2[PASS_TILE]
constexpr int P_BYTES = P_STAGE + 8 * PASS_TILE;
static_assert(P_BYTES >= 4 * PASS_LOCAL_G, "group counts fit the pool");
static_assert(P_BYTES - P_STAGE >= 16 * OWN_CAP + 8 * PASS_THREADS,
              "owned fields and run-start fields fit the staging area");
static_assert(P_STAGE >= 4 * PASS_LOCAL_G, "owned fields do not overlap the group counts");

// The deferred per-group plan writes of a block that owns at most OWN_CAP
// groups (their fields were left in `oex` by pass_local_plan).
__device__ void pass_owned_writes(const State &st, const Scratch &sc, const int4 *oex, int own_n,
                                  int32_t po0, int32_t c00, int32_t nl, int32_t seq, int mode,
                                  int32_t workers) {
    const int lo = (int)((int64_t)blockIdx.x * st.G / gridDim.x);
    for (int i = threadIdx.x; i < own_n; i += PASS_THREADS) {
        const int g = lo + i;
        const int4 e = oex[i];
        const int ex[PLAN_FIELDS] = {e.x, e.y & 0xffff, e.y >> 16};
        sc.lpre[g] = ex[0];
        if (e.z > 0) {
            const bool pre = i == (int)threadIdx.x;
            plan_group(st, sc, g, e.z, ex, pre ? po0 : st.pos[g], pre ? c00 : st.cnt[g], nl, seq,
                       mode, workers);
        }
    }
}

// Multisplit pass.  LOCAL: the plan is computed in the block (above) and
// bucket ids come from LDS; otherwise they are read from the plan's global
// per-group buckets.
// The multisplit of one tile whose keys, values and bucket ids (NB: none)
// are in registers: ranks inside each wave's chunk, tile-wide bucket
// offsets, the reordered tile written back contiguously and its row of
// bucket starts.  `after_clear` runs after the first barrier,
// `before_stores` before the first global store.  The LDS arrays are the
// caller's.
template <int NBM, int LEADB, typename F, typename H>
__device__ __forceinline__ void pass_split(const int32_t (&key)[PASS_ROUNDS],
                                           const int32_t (&val)[PASS_ROUNDS],
                                           const int32_t (&bk)[PASS_ROUNDS],
                                           int32_t (&lr)[PASS_ROUNDS], int NB, int64_t base,
                                           int tile_n, int tile, const Scratch &sc,
                                           uint16_t *wcp, int2 *stage, int32_t *ts, int *red,
                                           uint8_t *leadp, F &&after_clear, H &&before_stores) {
    static_assert(NBM % 2 == 0, "per-wave counter rows are cleared as 32-bit pairs");
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    uint16_t (*wc)[NBM] = reinterpret_cast<uint16_t (*)[NBM]>(wcp);
    // clear the per-wave counters two at a time, row by row (no division by
    // NB; a row may be cleared one entry past NB, which NB_MAX leaves room for)
    for (int p = tid; 2 * p < NB; p += PASS_THREADS)
#pragma unroll
        for (int w = 0; w < PASS_WAVES; ++w) reinterpret_cast<uint32_t *>(wc[w])[p] = 0;
    __syncthreads();
    after_clear();
    phase_mark(sc, PHASE_PASS, 1);
    // The lanes of a round that share a bucket elect one of them: each
    // writes its lane id into the wave's table at its bucket and, after a
    // wave-scope release/acquire, reads the entry back, so all of them read
    // the same surviving id (the accesses are wave-scope atomics: lanes race
    // on the entry by design, and a plain read could be folded into the
    // lane's own write).  Matching that 6-bit id takes 6 ballots instead of
    // one per bit of the bucket id.
    uint8_t *lead = leadp + wave * LEADB;
#pragma unroll
    for (int r = 0; r < PASS_ROUNDS; ++r) {
        const int b = bk[r];
        const bool valid = (unsigned)b < (unsigned)NB;
        if (valid)
            __hip_atomic_store(lead + b, (uint8_t)lane, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WAVEFRONT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int L = valid ? (int)__hip_atomic_load(lead + b, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WAVEFRONT)
                            : 0;
        const uint64_t m = match_lane_id(valid, L);
        if (valid) {
            const int below = lanes_below(m);
            const int c = wc[wave][b];
            lr[r] = c + below;
            if (below == 0) wc[wave][b] = (uint16_t)(c + __popcll(m));
        }
    }
    __syncthreads();
    phase_mark(sc, PHASE_PASS, 2);
    // per bucket: tile count, and each wave's offset inside the bucket
    for (int b = tid; b < NB; b += PASS_THREADS) {
        int s = 0;
#pragma unroll
        for (int w = 0; w < PASS_WAVES; ++w) {
            const int c = wc[w][b];
            wc[w][b] = (uint16_t)s;
            s += c;
        }
        ts[b] = s;
    }
    __syncthreads();
    block_excl_scan_array(ts, NB, red);
    phase_mark(sc, PHASE_PASS, 3);
#pragma unroll
    for (int r = 0; r < PASS_ROUNDS; ++r) {
        const int b = bk[r];
        if ((unsigned)b < (unsigned)NB) {
            const int slot = ts[b] + wc[wave][b] + lr[r];
            stage[slot] = make_int2(key[r], val[r]);
            if (sc.sidx)  // per-tuple results: where each staged tuple came from
                sc.sidx[base + slot] = (int32_t)(base + wave * (PASS_TILE / PASS_WAVES) + r * 64 + lane);
        }
    }
    __syncthreads();
    // the staged tuples (those of a bucket; fewer than the tile's when some
    // were dropped), two per 16-byte store (the tile starts 32 KB-aligned;
    // an odd last tuple is stored alone)
    before_stores();
    // (fixed trip counts, stores predicated: the number of stores in flight
    // is then known where later loads are waited for)
    const int kept = ts[NB];
    int2 *dst = sc.sdat + base;
    const int4 *st4 = reinterpret_cast<const int4 *>(stage);
    int4 *dst4 = reinterpret_cast<int4 *>(dst);
#pragma unroll
    for (int j = 0; j < PASS_TILE / 2 / PASS_THREADS; ++j) {
        const int i = tid + j * PASS_THREADS;
        if (i < kept / 2) dst4[i] = st4[i];
    }
    if ((kept & 1) && tid == 0) dst[kept - 1] = stage[kept - 1];
    int32_t *row = sc.rowstart + (int64_t)tile * (NB + 1);
#pragma unroll
    for (int j = 0; j < (NBM + PASS_THREADS) / PASS_THREADS; ++j) {
        const int b = tid + j * PASS_THREADS;
        if (b <= NB) row[b] = ts[b];
    }
    phase_mark(sc, PHASE_PASS, 4);
}

// One tile (`tile`: its index in the sub-batch) per block.
template <bool LOCAL>
__device__ __forceinline__ void pass_tile(const int32_t *__restrict__ keys,
                                          const int32_t *__restrict__ values, int64_t n,
                                          const State &st, const Scratch &sc, int32_t seq,
                                          int mode, int32_t workers, int tile) {
    // per-wave bucket counters and the reordered tile; during an in-block
    // plan the same bytes hold the group counts
    __shared__ __align__(16) char pool[P_BYTES];
    __shared__ int32_t ts[NB_MAX + 1];
    __shared__ int red[PASS_WAVES];
    // group -> bucket ids during an in-block plan; then, in both variants,
    // one LEAD-byte leader table per wave for the multisplit
    __shared__ __align__(16) uint16_t gbk[PASS_LOCAL_G];
    __shared__ int pred[2 * PASS_WAVES];
    __shared__ unsigned long long ptop[2 * PASS_WAVES];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int64_t base = (int64_t)tile * PASS_TILE;
    const int tile_n = (int)min((int64_t)PASS_TILE, n - base);
    phase_mark(sc, PHASE_PASS, 0);
    int32_t key[PASS_ROUNDS], val[PASS_ROUNDS], bk[PASS_ROUNDS], lr[PASS_ROUNDS];
    // Raw keys, loaded unconditionally from an index clamped into the batch
    // (n >= 1), so that no load waits on another; lanes past n are masked
    // where the keys are first used, and the group view is applied there.
    auto load_tile = [&]() {
#pragma unroll
        for (int r = 0; r < PASS_ROUNDS; ++r) {
            const int64_t i = min(base + wave * (PASS_TILE / PASS_WAVES) + r * 64 + lane, n - 1);
            key[r] = keys[i];
            val[r] = values[i];
        }
    };
    int NB;
    int own_n = 0;
    int32_t po0 = 0, c00 = 0, nl = 0;
    if (LOCAL) {
        NB = pass_local_plan(st, sc, seq, mode, workers, gbk, reinterpret_cast<int32_t *>(pool),
                             reinterpret_cast<int4 *>(pool + P_STAGE), pred, ptop, own_n, po0,
                             c00, nl, load_tile);
        if (NB < 0) return;
        if (NB > LEAD) {  // no plan makes this many buckets
            if (tid == 0) atomicOr(sc.fault, FAULT_BUCKETS);
            return;
        }
#pragma unroll
        for (int r = 0; r < PASS_ROUNDS; ++r) {
            const int64_t i = base + wave * (PASS_TILE / PASS_WAVES) + r * 64 + lane;
            key[r] = view_key(key[r], sc.kmod, st.G);
            bk[r] = (i < n && (uint32_t)key[r] < (uint32_t)st.G) ? gbk[key[r]] : NB;
            lr[r] = 0;
        }
    } else {
        load_tile();
        const PlanTotals t = *sc.tot;
        if (t.status) return;
        NB = t.n_buckets;
        if (NB > LEAD) {  // no plan makes this many buckets
            if (tid == 0) atomicOr(sc.fault, FAULT_BUCKETS);
            return;
        }
#pragma unroll
        for (int r = 0; r < PASS_ROUNDS; ++r) {
            const int64_t i = base + wave * (PASS_TILE / PASS_WAVES) + r * 64 + lane;
            key[r] = view_key(key[r], sc.kmod, st.G);
            bk[r] = (i < n) ? sc.bucket[key[r]] : NB;
            lr[r] = 0;
        }
    }
    pass_split<NB_MAX, LEAD>(
        key, val, bk, lr, NB, base, tile_n, tile, sc, reinterpret_cast<uint16_t *>(pool + P_WC),
        reinterpret_cast<int2 *>(pool + P_STAGE), ts, red, reinterpret_cast<uint8_t *>(gbk),
        [&]() {
            // the plan's per-group writes (fields in the staging area, which
            // is written only after two more barriers)
            if (LOCAL && own_n > 0)
                pass_owned_writes(st, sc, reinterpret_cast<const int4 *>(pool + P_STAGE), own_n,
                                  po0, c00, nl, seq, mode, workers);
        },
        [] {});
}

template <bool LOCAL>
__global__ __launch_bounds__(PASS_THREADS) void k_pass(const int32_t *__restrict__ keys,
                                                       const int32_t *__restrict__ values,
                                                       int64_t n, State st, Scratch sc,
                                                       int32_t seq, int mode, int32_t workers) {
    if (sc.seqp) seq = *sc.seqp;  // captured for replay: the argument would be stale
    pass_tile<LOCAL>(keys, values, n, st, sc, seq, mode, workers, (int)blockIdx.x);
}

// ------------------------------------------------------------- k_update --

__device__ __forceinline__ void emit_one(const Out &out, int32_t j, int32_t g, int64_t s,
                                         int32_t c) {
    if (out.ids) global_ptr(out.ids)[j] = g;
    if (out.sums) global_ptr(out.sums)[j] = s;
    if (out.counts) global_ptr(out.counts)[j] = c;
    if (out.avgs) global_ptr(out.avgs)[j] = (double)s / (double)c;
}

__device__ __forceinline__ void trace_record(int64_t *trace, int rec, unsigned long long t0,
                                             int64_t tuples, int64_t items) {
    if (!trace || threadIdx.x != 0) return;
    const unsigned long long t1 = wall_clock64();
    const uint32_t hwid = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4);
    const uint32_t xcc = __builtin_amdgcn_s_getreg((15 << 11) | (0 << 6) | 20);
    int64_t *r = trace + 6 * (int64_t)rec;
    r[0] = hwid;
    r[1] = xcc;
    r[2] = (int64_t)t0;
    r[3] = (int64_t)t1;
    r[4] = tuples;
    r[5] = items;
}

// LDS layout of the balanced per-group phase (bytes).
constexpr int U_RS = 0;                                  // i32[PASS_TILES_MAX]
constexpr int U_RP = U_RS + 4 * PASS_TILES_MAX;          // i32[PASS_TILES_MAX + 1]
constexpr int U_EK = U_RP + 4 * (PASS_TILES_MAX + 4);    // i32[LIGHT_CAP] keys
constexpr int U_EV = U_EK + 4 * LIGHT_CAP;               // i32[LIGHT_CAP] values
constexpr int U_PZ = U_EV + 4 * LIGHT_CAP;               // i16[LIGHT_CAP] group start in bucket
constexpr int U_LR = U_PZ + 2 * LIGHT_CAP;               // u16[LIGHT_CAP] rank inside wave chunk
                                                         // (first: u8 run of each position)
constexpr int U_HD = U_LR + 2 * LIGHT_CAP;               // i16[LIGHT_CAP] tuple of rank 0
constexpr int U_CW = U_HD + 2 * LIGHT_CAP;               // u16[UPD_WAVES][LIGHT_CAP]
constexpr int UPD_WAVES = UPD_THREADS / 64;
constexpr int U_ACC = U_CW + 2 * UPD_WAVES * LIGHT_CAP;  // i64[LIGHT_CAP] sum deltas
// a light bucket whose groups span at most LIGHT_SPAN ids keeps their
// staged-range starts and old ring pointers in LDS
constexpr int LIGHT_SPAN = 768;
static_assert(LIGHT_SPAN % UPD_THREADS == 0, "whole groups per thread");
constexpr int U_KLP = U_ACC + 8 * LIGHT_CAP;             // i32[LIGHT_SPAN + 1]
constexpr int U_KPO = U_KLP + 4 * (LIGHT_SPAN + 4);      // i32[LIGHT_SPAN]
constexpr int U_BYTES = U_KPO + 4 * LIGHT_SPAN;
static_assert(LIGHT_CAP <= 32768, "16-bit positions");
static_assert(PASS_TILES_MAX <= 256, "8-bit run indices");
static_assert(LIGHT_CAP % UPD_THREADS == 0, "whole positions per thread");

// The tuples of light bucket [a, z) (groups packed by the plan, fewer than
// LIGHT_CAP tuples, runs already in rs/rp), read in arrival order into LDS
// (ek, ev, pz) and ranked: each wave takes a contiguous chunk; in every
// 64-lane round the lanes holding the same group find each other with
// ballots over the group's start position, so a tuple's rank among its
// group's earlier tuples is exact and stable (light_rank_of).  Returns false
// for an empty bucket or a malformed plan (flagged).
// IN_LDS: the bucket's groups span at most LIGHT_SPAN ids and their
// staged-range starts were prefetched into LDS (a template parameter, so
// that each read is a plain LDS or global load, never a generic one that the
// compiler must wait on as both).
template <bool IN_LDS>
__device__ bool light_rank(int32_t a, int32_t z, int size, int tiles, const Scratch &sc,
                           char *smem) {
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int32_t *rs = reinterpret_cast<const int32_t *>(smem + U_RS);
    const int32_t *rp = reinterpret_cast<const int32_t *>(smem + U_RP);
    int32_t *ek = reinterpret_cast<int32_t *>(smem + U_EK);
    int32_t *ev = reinterpret_cast<int32_t *>(smem + U_EV);
    int16_t *pz = reinterpret_cast<int16_t *>(smem + U_PZ);
    uint16_t *lr = reinterpret_cast<uint16_t *>(smem + U_LR);
    int16_t *hd = reinterpret_cast<int16_t *>(smem + U_HD);
    uint16_t *cw = reinterpret_cast<uint16_t *>(smem + U_CW);
    long long *acc = reinterpret_cast<long long *>(smem + U_ACC);
    const int32_t *klp = reinterpret_cast<const int32_t *>(smem + U_KLP);
    constexpr bool in_lds = IN_LDS;
    // staged-range start of g (relative to the bucket)
    auto lp = [&](int32_t g) { return in_lds ? klp[g - a] : sc.lpre[g]; };
    const int32_t s0 = lp(a);
    if (size <= 0) return false;
    if (size > LIGHT_CAP || lp(z) - s0 != size) {
        if (tid == 0) atomicOr(sc.fault, FAULT_LIGHT_SIZE);
        return false;
    }
    // run (tile) of every bucket position, so the gather below needs one
    // LDS read instead of a binary search over the runs: mark each
    // non-empty run's tile at its first position, then a running maximum
    // over the positions (tile ids grow with position).  lr is free until
    // the ranks; the caller cleared it before the barrier that stored the
    // runs.
    uint8_t *rt = reinterpret_cast<uint8_t *>(lr);
    {
        constexpr int PPT = LIGHT_CAP / UPD_THREADS;
        for (int r = tid; r < tiles; r += blockDim.x)
            if (rp[r + 1] > rp[r]) rt[rp[r]] = (uint8_t)r;
        __syncthreads();
        int loc[PPT], m = 0;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int p = tid * PPT + j;
            m = max(m, p < size ? (int)rt[p] : 0);
            loc[j] = m;
        }
        const int incl = wave_incl_max(m);
        int *wred = reinterpret_cast<int *>(ev);  // ev is filled only below
        if (lane == 63) wred[wv] = incl;
        __syncthreads();
        int before = __shfl_up(incl, 1, 64);
        if (lane == 0) before = 0;
        for (int w = 0; w < wv; ++w) before = max(before, wred[w]);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int p = tid * PPT + j;
            if (p < size) rt[p] = (uint8_t)max(before, loc[j]);
        }
        __syncthreads();
    }
    // all of this thread's gathers are issued before any is used
    constexpr int SPT = LIGHT_CAP / UPD_THREADS;
    int2 st_e[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int p = tid + j * UPD_THREADS;
        st_e[j] = make_int2(a, 0);
        if (p < size) {
            const int r = rt[p];
            st_e[j] = sc.sdat[rs[r] + (p - rp[r])];
        }
    }
    // Without the LDS copy, each tuple's group bounds in the staged order
    // are read from global memory all at once, before any is used (a key
    // outside the bucket reads group a's, and is flagged below).
    int32_t l0v[SPT], l1v[SPT];
    if constexpr (!IN_LDS) {
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            const int32_t g = st_e[j].x;
            const int32_t gc = g >= a && g < z ? g : a;
            l0v[j] = lp(gc);
            l1v[j] = lp(gc + 1);
        }
    }
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int p = tid + j * UPD_THREADS;
        if (p >= size) continue;
        const int2 e = st_e[j];
        const int32_t g = e.x;
        int32_t p0 = -1;
        if (g >= a && g < z) {
            const int32_t l0 = IN_LDS ? lp(g) : l0v[j];
            if ((IN_LDS ? lp(g + 1) : l1v[j]) > l0) p0 = l0 - s0;
        }
        if (p0 < 0 || p0 >= size) {  // impossible for a well-formed plan
            atomicOr(sc.fault, FAULT_LIGHT_SIZE);
            p0 = -1;
        }
        ek[p] = g;
        ev[p] = e.y;
        pz[p] = (int16_t)p0;
        hd[p] = -1;
    }
    for (int i = tid; i < size; i += UPD_THREADS)
#pragma unroll
        for (int w = 0; w < UPD_WAVES; ++w) cw[w * LIGHT_CAP + i] = 0;
    __syncthreads();
    phase_mark(sc, PHASE_UPDATE, 2);
    // ranks inside each wave's chunk of the arrival order
    const int chunk = (size + UPD_WAVES - 1) / UPD_WAVES;
    const int c0 = min(size, wv * chunk), c1 = min(size, c0 + chunk);
    uint16_t *mycw = cw + wv * LIGHT_CAP;
    // The lanes of a round that hold one group elect one of them through a
    // per-wave byte table indexed by the group's start position (in `acc`,
    // which is free until the ring update and cleared after the ranks), as
    // the reorder pass does for buckets: 6 ballots over the elected lane id.
    uint8_t *lead = reinterpret_cast<uint8_t *>(acc) + wv * LIGHT_CAP;
    for (int r0 = c0; r0 < c1; r0 += 64) {
        const int p = r0 + lane;
        const bool valid = p < c1 && pz[p] >= 0;
        const int p0 = valid ? pz[p] : 0;
        if (valid)
            __hip_atomic_store(lead + p0, (uint8_t)lane, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WAVEFRONT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int L = valid ? (int)__hip_atomic_load(lead + p0, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WAVEFRONT)
                            : 0;
        const uint64_t m = match_lane_id(valid, L);
        if (valid) {
            const int below = lanes_below(m);
            const int c = mycw[p0];
            lr[p] = (uint16_t)(c + below);
            if (below == 0) mycw[p0] = (uint16_t)(c + __popcll(m));
        }
    }
    __syncthreads();
    // each group's count per wave -> the wave's offset inside the group
    // (and the sum deltas cleared: the leader tables are done with)
    for (int i = tid; i < size; i += blockDim.x) {
        acc[i] = 0;
        int sacc = 0;
#pragma unroll
        for (int w = 0; w < UPD_WAVES; ++w) {
            const int c = cw[w * LIGHT_CAP + i];
            cw[w * LIGHT_CAP + i] = (uint16_t)sacc;
            sacc += c;
        }
    }
    __syncthreads();
    return true;
}

// The rank of the tuple at bucket position p among its group's tuples
// (arrival order), after light_rank: its wave's offset inside the group
// plus its rank inside the wave's chunk.
__device__ __forceinline__ int32_t light_rank_of(const char *smem, int size, int p) {
    const int16_t *pz = reinterpret_cast<const int16_t *>(smem + U_PZ);
    const uint16_t *lr = reinterpret_cast<const uint16_t *>(smem + U_LR);
    const uint16_t *cw = reinterpret_cast<const uint16_t *>(smem + U_CW);
    const int chunk = (size + UPD_WAVES - 1) / UPD_WAVES;
    int w = 0;  // the wave whose chunk holds p
#pragma unroll
    for (int k = 1; k < UPD_WAVES; ++k) w += p >= k * chunk ? 1 : 0;
    return cw[w * LIGHT_CAP + pz[p]] + lr[p];
}

// Light bucket b: groups [bstart[b], bstart[b+1]) packed by the plan, fewer
// than LIGHT_CAP tuples, ranked by light_rank.  Every tuple among its
// group's last W goes to ring slot (pos + rank) mod W and the group's sum
// gains (new value - value overwritten).
template <bool IN_LDS>
__device__ int light_bucket(int32_t a, int32_t z, int size, int tiles, const State &st,
                            const Scratch &sc, const Out &out, char *smem) {
    if (!light_rank<IN_LDS>(a, z, size, tiles, sc, smem)) return 0;
    const int tid = threadIdx.x;
    int32_t *ek = reinterpret_cast<int32_t *>(smem + U_EK);
    int32_t *ev = reinterpret_cast<int32_t *>(smem + U_EV);
    int16_t *pz = reinterpret_cast<int16_t *>(smem + U_PZ);
    uint16_t *lr = reinterpret_cast<uint16_t *>(smem + U_LR);
    int16_t *hd = reinterpret_cast<int16_t *>(smem + U_HD);
    uint16_t *cw = reinterpret_cast<uint16_t *>(smem + U_CW);
    long long *acc = reinterpret_cast<long long *>(smem + U_ACC);
    const int32_t *klp = reinterpret_cast<const int32_t *>(smem + U_KLP);
    const int32_t *kpo = reinterpret_cast<const int32_t *>(smem + U_KPO);
    constexpr bool in_lds = IN_LDS;
    // (the per-group arrays as global pointers: held in a struct, they would
    // otherwise be accessed as generic memory)
    const auto lpre = global_ptr(sc.lpre), pold = global_ptr(sc.pold);
    const auto ncnt = global_ptr(sc.ncnt), tidx = global_ptr(sc.tidx);
    const auto gsm = global_ptr(st.sum);
    const auto ring = global_ptr(st.ring);
    auto lp = [&](int32_t g) { return in_lds ? klp[g - a] : lpre[g]; };
    auto po = [&](int32_t g) { return in_lds ? kpo[g - a] : pold[g]; };
    const int32_t s0 = lp(a);
    const int chunk = (size + UPD_WAVES - 1) / UPD_WAVES;
    constexpr int SPT = LIGHT_CAP / UPD_THREADS;
    const int32_t W = st.W;
    phase_mark(sc, PHASE_UPDATE, 3);
    // the touched groups' sums, counts and output slots are loaded now, so
    // that their latency overlaps the ring update below
    constexpr int GPT = LIGHT_SPAN / UPD_THREADS;
    int64_t gsum[GPT];
    int32_t gcnt[GPT], gtix[GPT];
    // (every load is issued, from group a where the thread has no touched
    // group, and the values are selected afterwards: a load under a
    // divergent branch would be waited on before the next one is issued)
    if (in_lds) {
#pragma unroll
        for (int j = 0; j < GPT; ++j) {
            const int32_t g = a + tid + j * UPD_THREADS;
            const bool t = g < z && klp[g - a + 1] > klp[g - a];
            const int32_t gl = t ? g : a;
            gsum[j] = gsm[gl];  // (raw: read only for a touched group, below)
            gcnt[j] = ncnt[gl];
            gtix[j] = tidx[gl];
        }
    }
    // ring update: every survivor's old value is loaded before any store
    // (unconditionally, from the ring's first cell where there is none to
    // read, so that the loads are in flight together)
    int64_t cells[SPT];  // ring index of the slot a survivor takes (-1: none)
    int32_t olds[SPT];
    bool keep[SPT];  // the old value counts: a survivor whose window is not replaced
    // (without the LDS copy, each position's group bounds and old ring
    // pointer are read from global memory all at once, group a where the
    // position has none)
    int32_t kq[SPT], oq[SPT];
    if constexpr (!IN_LDS) {
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            const int p = tid + j * UPD_THREADS;
            const int32_t e = ek[p];  // (read apart from the select: p < LIGHT_CAP)
            const int32_t g = p < size && pz[p] >= 0 ? e : a;
            kq[j] = lp(g + 1) - lp(g);
            oq[j] = po(g);
        }
    }
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int p = tid + j * UPD_THREADS;
        cells[j] = -1;
        keep[j] = false;
        if (p >= size) continue;
        const int p0 = pz[p];
        if (p0 < 0) continue;
        int w = 0;  // the wave whose chunk holds p
#pragma unroll
        for (int k = 1; k < UPD_WAVES; ++k) w += p >= k * chunk ? 1 : 0;
        const int32_t g = ek[p];
        const int32_t rank = cw[w * LIGHT_CAP + p0] + lr[p];
        const int32_t kg = IN_LDS ? lp(g + 1) - lp(g) : kq[j];
        if (rank == 0) hd[p0] = (int16_t)p;
        const int32_t need = kg < W ? kg : W;
        if (rank >= kg - need && rank < kg) {
            const uint32_t slot =
                ((uint32_t)(IN_LDS ? po(g) : oq[j]) + (uint32_t)rank) % (uint32_t)W;
            cells[j] = (int64_t)g * W + slot;
            keep[j] = kg < W;
        }
    }
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int32_t o = ring[cells[j] >= 0 ? cells[j] : 0];
        olds[j] = keep[j] ? o : 0;
    }
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        if (cells[j] < 0) continue;
        const int p = tid + j * UPD_THREADS;
        const int32_t v = ev[p];
        ring[cells[j]] = v;
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc[pz[p]]),
                  (unsigned long long)((long long)v - (long long)olds[j]));
    }
    __syncthreads();
    phase_mark(sc, PHASE_UPDATE, 4);
    if (in_lds) {
#pragma unroll
        for (int j = 0; j < GPT; ++j) {
            const int32_t g = a + tid + j * UPD_THREADS;
            if (g < z && klp[g - a + 1] > klp[g - a]) {
                // a group with at least W tuples here has its window
                // replaced whole: its new sum is the survivors' sum alone
                const int64_t s = (klp[g - a + 1] - klp[g - a] < W ? gsum[j] : 0) +
                                  acc[klp[g - a] - s0];
                gsm[g] = s;
                if (out.n_touched) emit_one(out, gtix[j], g, s, gcnt[j]);
            }
        }
    } else {
        // the touched groups' state, all read before any is used (group a
        // where a position heads no group)
        int32_t gh[SPT], kh[SPT], th[SPT], nh[SPT];
        int64_t sh[SPT];
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            const int i = tid + j * UPD_THREADS;
            gh[j] = i < size && hd[i] >= 0 ? ek[hd[i]] : -1;
            const int32_t g = gh[j] >= 0 ? gh[j] : a;
            kh[j] = lp(g + 1) - lp(g);
            sh[j] = gsm[g];
            th[j] = tidx[g];
            nh[j] = ncnt[g];
        }
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            const int i = tid + j * UPD_THREADS;
            const int32_t g = gh[j];
            if (g >= 0) {
                const int64_t s = (kh[j] >= W ? 0 : sh[j]) + acc[i];
                gsm[g] = s;
                if (out.n_touched) emit_one(out, th[j], g, s, nh[j]);
            }
        }
    }
    __syncthreads();
    return size;
}

// Heavy bucket (one group, size >= HEAVY_MIN tuples): only its last
// min(size, W) tuples survive; they are read straight from their runs.
__device__ int heavy_bucket(int32_t g, int32_t pold_g, int size, int tiles, const State &st,
                            const Scratch &sc, const Out &out, char *smem, long long *red_ll) {
    const int tid = threadIdx.x;
    const int32_t *rs = reinterpret_cast<const int32_t *>(smem + U_RS);
    const int32_t *rp = reinterpret_cast<const int32_t *>(smem + U_RP);
    const int32_t W = st.W;
    const int32_t need = size < W ? size : W;
    const bool full = size >= W;
    const uint32_t po = (uint32_t)pold_g;
    // loaded early, by every thread (one address), so that no wait on them
    // comes before the survivors' loads are issued
    const int64_t gsum_old = st.sum[g];
    const int32_t gcnt = sc.ncnt[g], gtix = sc.tidx[g];
    long long acc = 0;
    // (a run table as in light buckets would cost one thread a serial loop
    // over a hot group's whole run in the last tile; a binary search per
    // survivor is cheaper here)
    // HU survivors per thread at a time, all loaded before any store
    constexpr int HU = 4;
    for (int p0 = size - need + tid; p0 < size; p0 += HU * UPD_THREADS) {
        int32_t vals[HU], olds[HU];
        int32_t *cells[HU];
        // positions past the bucket are clamped onto its last one, so every
        // load is issued unconditionally; only real positions store
#pragma unroll
        for (int u = 0; u < HU; ++u) {
            const int p = p0 + u * UPD_THREADS;
            const int pc = p < size ? p : size - 1;
            const int r = upper_run(rp, tiles, pc);
            vals[u] = sc.sdat[rs[r] + (pc - rp[r])].y;
            const uint32_t slot = (po + (uint32_t)pc) % (uint32_t)W;
            int32_t *cell = st.ring + (int64_t)g * W + slot;
            cells[u] = p < size ? cell : nullptr;
            olds[u] = *cell;  // (dropped below for a window replaced whole)
        }
#pragma unroll
        for (int u = 0; u < HU; ++u)
            if (cells[u]) {
                *cells[u] = vals[u];
                acc += (long long)vals[u] - (full ? 0LL : (long long)olds[u]);
            }
    }
    const long long delta = block_sum_ll(acc, red_ll);
    if (tid == 0) {
        const int64_t s = (full ? 0 : gsum_old) + delta;  // a window replaced whole restarts at 0
        st.sum[g] = s;
        if (out.n_touched) emit_one(out, gtix, g, s, gcnt);
    }
    __syncthreads();
    return need;
}

// Histogram of the next batch of a pipelined call, run by the last
// nh.blocks workgroups of an update launch (so that it costs no launch of
// its own): UPD_THREADS threads over FH_TILE consecutive keys.  A tile holds
// fewer than 2^16 keys, so the LDS counters are 16-bit halves of words
// (key k in word k/2), and the group counts fit the update's LDS.
constexpr int FH_KPT = 32;
constexpr int FH_TILE = UPD_THREADS * FH_KPT;
static_assert(FH_TILE < 65536, "16-bit counters");
static_assert(PASS_LOCAL_G / 2 * 4 <= U_BYTES, "packed counters fit the update's LDS");

__device__ void fused_hist(const NextHist &h, int hb, int nhb, int32_t G, uint32_t *cw) {
    const int tid = threadIdx.x;
    const int32_t hot0 = h.sc.hot[0], hot1 = h.sc.hot[1];
    const int words = (G + 1) / 2;
    for (int w = tid; w < words; w += UPD_THREADS) cw[w] = 0;
    const int64_t base = (int64_t)hb * FH_TILE;
    int32_t v[FH_KPT];
#pragma unroll
    for (int j = 0; j < FH_KPT / 4; ++j) {
        const int64_t i = base + 4 * ((int64_t)j * UPD_THREADS + tid);
        if (h.vec && i + 3 < h.n) {
            const int4 x = *reinterpret_cast<const int4 *>(h.keys + i);
            v[4 * j] = x.x; v[4 * j + 1] = x.y; v[4 * j + 2] = x.z; v[4 * j + 3] = x.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[4 * j + e] = (i + e < h.n) ? h.keys[i + e] : 0;
        }
    }
    if (h.sc.kmod) {
#pragma unroll
        for (int j = 0; j < FH_KPT; ++j) v[j] = view_key(v[j], h.sc.kmod, G);
    }
    __syncthreads();
    int bad = 0, c0 = 0, c1 = 0;
#pragma unroll
    for (int j = 0; j < FH_KPT / 4; ++j) {
        const int64_t i = base + 4 * ((int64_t)j * UPD_THREADS + tid);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (i + e >= h.n) continue;
            const int32_t key = v[4 * j + e];
            if (key < 0 || key >= G) bad = 1;
            else if (key == hot0) ++c0;
            else if (key == hot1) ++c1;
            else atomicAdd(&cw[key >> 1], (key & 1) ? 65536u : 1u);
        }
    }
    c0 = wave_total(wave_incl_add(c0));
    c1 = wave_total(wave_incl_add(c1));
    if (lane_id() == 0) {
        if (c0) atomicAdd(&cw[hot0 >> 1], (uint32_t)c0 << (16 * (hot0 & 1)));
        if (c1) atomicAdd(&cw[hot1 >> 1], (uint32_t)c1 << (16 * (hot1 & 1)));
    }
    if (__syncthreads_or(bad)) {
        if (tid == 0) atomicExch(h.sc.bad, h.sc.seqp ? *h.sc.seqp + 1 : h.seq);
    }
    // staggered flush, as in k_hist_small
    const int off = (int)(((int64_t)hb * words / nhb) & ~31);
    for (int i = tid; i < words; i += UPD_THREADS) {
        const int w = i + off < words ? i + off : i + off - words;
        const uint32_t c = cw[w];
        if (c & 0xffff) atomicAdd(&h.sc.k[2 * w], (int32_t)(c & 0xffff));
        if (c >> 16) atomicAdd(&h.sc.k[2 * w + 1], (int32_t)(c >> 16));
    }
}

__global__ __launch_bounds__(UPD_THREADS) void k_update_balanced(State st, Scratch sc, int tiles,
                                                                 Out out, NextHist nh) {
    __shared__ __align__(16) char smem[U_BYTES];
    __shared__ int red[UPD_THREADS / 64];
    __shared__ long long red_ll[UPD_THREADS / 64];
    const unsigned long long t0 = wall_clock64();
    // the next batch's histogram takes the first nh.blocks workgroups (they
    // are dispatched first and finish early); the update takes the rest
    const int ug = (int)gridDim.x - nh.blocks;
    if ((int)blockIdx.x < nh.blocks) {
        fused_hist(nh, (int)blockIdx.x, nh.blocks, (int32_t)st.G,
                   reinterpret_cast<uint32_t *>(smem));
        return;
    }
    const int ub = (int)blockIdx.x - nh.blocks;  // workgroup index within the update
    const PlanTotals t = *sc.tot;
    if (t.status) {
        if (ub == 0 && threadIdx.x == 0 && out.n_touched) *out.n_touched = t.status;
        return;
    }
    if (ub == 0 && threadIdx.x == 0 && out.n_touched) *out.n_touched = t.n_touched;
    int64_t tuples = 0, items = 0;
    const int NB = t.n_buckets;
    int32_t *rs = reinterpret_cast<int32_t *>(smem + U_RS);
    int32_t *rp = reinterpret_cast<int32_t *>(smem + U_RP);
    phase_mark(sc, PHASE_UPDATE, 0);
    int32_t *klp = reinterpret_cast<int32_t *>(smem + U_KLP);
    int32_t *kpo = reinterpret_cast<int32_t *>(smem + U_KPO);
    // Workgroups are dispatched to the XCDs round-robin (workgroup i on XCD
    // i mod XCDS); each XCD takes one contiguous range of buckets, so the
    // cache lines that neighbouring buckets share in the staged tiles and
    // their rows of bucket starts stay in one XCD's L2.
    const int xcd = ub % XCDS, per_xcd = ug / XCDS;
    const int span = (NB + XCDS - 1) / XCDS;
    const int b_lo = xcd * span, b_hi = min(NB, b_lo + span);
    const int first = ub / XCDS < per_xcd ? b_lo + ub / XCDS : NB;
    for (int b = first; b < b_hi; b += per_xcd) {
        const bool light = b < t.n_light_buckets;
        int32_t a = 0, z = 0, g = 0;
        if (light) {
            a = sc.bstart[b];
            z = sc.bstart[b + 1];
        } else {
            g = sc.hkey[b - t.n_light_buckets];
        }
        // The bucket's runs, and (a light bucket of at most LIGHT_SPAN
        // groups) its groups' staged-range starts and old ring pointers for
        // LDS: every load is issued before any is waited on (indexes
        // clamped into the bucket's groups, values kept only where in range).
        RunRows<UPD_THREADS> rr;
        runs_load<UPD_THREADS>(sc, b, NB, tiles, rr);
        const int32_t pold_g = sc.pold[light ? a : g];  // read by a heavy bucket only
        constexpr int KPT = LIGHT_SPAN / UPD_THREADS;
        int32_t pl[KPT + 1], pp[KPT];
        const int m = z - a;  // groups of a light bucket (at least 1)
        const bool pre = light && m <= LIGHT_SPAN;
        if (pre) {
#pragma unroll
            for (int j = 0; j <= KPT; ++j)
                pl[j] = sc.lpre[a + min((int)threadIdx.x + j * UPD_THREADS, m)];
#pragma unroll
            for (int j = 0; j < KPT; ++j)
                pp[j] = sc.pold[a + max(0, min((int)threadIdx.x + j * UPD_THREADS, m - 1))];
        }
        if (pre) {
#pragma unroll
            for (int j = 0; j <= KPT; ++j) {
                const int i = (int)threadIdx.x + j * UPD_THREADS;
                if (i <= m) klp[i] = pl[j];
                if (j < KPT && i < m) kpo[i] = pp[j];
            }
        }
        if (light)  // the light bucket's run table (LIGHT_CAP bytes) starts clear
            for (int i = threadIdx.x; i < LIGHT_CAP / 4; i += UPD_THREADS)
                reinterpret_cast<uint32_t *>(smem + U_LR)[i] = 0;
        const int size = runs_store<UPD_THREADS>(tiles, rr, rs, rp, red);
        if (b == first) phase_mark(sc, PHASE_UPDATE, 1);
        if (light)
            tuples += z - a <= LIGHT_SPAN
                          ? light_bucket<true>(a, z, size, tiles, st, sc, out, smem)
                          : light_bucket<false>(a, z, size, tiles, st, sc, out, smem);
        else
            tuples += heavy_bucket(g, pold_g, size, tiles, st, sc, out, smem, red_ll);
        // clear the bucket's histogram entries for the next sub-batch (the
        // buckets partition the touched groups)
        if (light)
            for (int i = threadIdx.x; i < z - a; i += blockDim.x) sc.k[a + i] = 0;
        else if (threadIdx.x == 0)
            sc.k[g] = 0;
        ++items;
    }
    phase_mark(sc, PHASE_UPDATE, 5);
    trace_record(sc.trace, ub, t0, tuples, items);
}

// Static assignment: worker w (one wave) owns groups [g0(w), g0(w+1)) and
// streams all of their tuples in arrival order, 64 at a time; lanes holding
// the same group find each other with ballots and a per-group counter gives
// ranks.  A worker's time grows with the tuples of its groups.
constexpr int S_RS = 0;                                                   // i32[4][T]
constexpr int S_RP = S_RS + 4 * STATIC_WORKERS_PER_WG * PASS_TILES_MAX;   // i32[4][T+1]
constexpr int S_CTR = S_RP + 4 * STATIC_WORKERS_PER_WG * (PASS_TILES_MAX + 1);
constexpr int S_ACC = S_CTR + 4 * STATIC_WORKERS_PER_WG * STATIC_KEYS_MAX + 16;
constexpr int S_BYTES = S_ACC + 8 * STATIC_WORKERS_PER_WG * STATIC_KEYS_MAX;

__device__ __forceinline__ int32_t static_first(int64_t w, int64_t G, int32_t workers) {
    return (int32_t)((w * G + workers - 1) / workers);
}

__global__ __launch_bounds__(UPD_THREADS) void k_update_static(State st, Scratch sc, int tiles,
                                                               int32_t workers, Out out) {
    __shared__ __align__(16) char smem[S_BYTES];
    __shared__ long long tend[STATIC_WORKERS_PER_WG];
    __shared__ long long tsum[STATIC_WORKERS_PER_WG];
    const unsigned long long t0 = wall_clock64();
    const PlanTotals t = *sc.tot;
    if (t.status) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && out.n_touched) *out.n_touched = t.status;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && out.n_touched) *out.n_touched = t.n_touched;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * STATIC_WORKERS_PER_WG + wv;
    const int NB = t.n_buckets;
    const int64_t G = st.G;
    const int32_t W = st.W;
    int32_t *rs = reinterpret_cast<int32_t *>(smem + S_RS) + wv * PASS_TILES_MAX;
    int32_t *rp = reinterpret_cast<int32_t *>(smem + S_RP) + wv * (PASS_TILES_MAX + 1);
    int32_t *ctr = reinterpret_cast<int32_t *>(smem + S_CTR) + wv * STATIC_KEYS_MAX;
    long long *acc = reinterpret_cast<long long *>(smem + S_ACC) + wv * STATIC_KEYS_MAX;
    int64_t tuples = 0;
    if (w < workers && w < NB) {
        // worker w's groups: a range, or its list under a Section 4 mapping
        int32_t g0 = 0, nk;
        const int32_t *list = nullptr;
        if (sc.wstart) {
            const int32_t a = sc.wstart[w];
            nk = sc.wstart[w + 1] - a;
            list = sc.wlist + a;
        } else {
            g0 = static_first(w, G, workers);
            nk = static_first(w + 1, G, workers) - g0;
        }
        if (nk > STATIC_KEYS_MAX) {
            if (lane == 0) atomicOr(sc.fault, FAULT_STATIC_KEYS);
        } else {
            for (int i = lane; i < nk; i += 64) {
                ctr[i] = 0;
                acc[i] = 0;
                sc.k[list ? list[i] : g0 + i] = 0;  // histogram, for the next sub-batch
            }
            // runs of bucket w, and a wave-wide exclusive scan of their sizes
            int carry = 0;
            for (int tb = 0; tb < tiles; tb += 64) {
                const int tt = tb + lane;
                int len = 0;
                if (tt < tiles) {
                    const int32_t *row = sc.rowstart + (int64_t)tt * (NB + 1);
                    const int32_t s = row[w], e = row[w + 1];
                    rs[tt] = tt * PASS_TILE + s;
                    len = e - s;
                }
                const int incl = wave_incl_add(len);
                if (tt < tiles) rp[tt] = carry + incl - len;
                carry += wave_total(incl);
            }
            if (lane == 0) rp[tiles] = carry;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int size = carry;
            tuples = size;
            for (int c0 = 0; c0 < size; c0 += 64) {
                const int p = c0 + lane;
                bool valid = p < size;
                int32_t g = list ? (nk ? list[0] : 0) : g0, v = 0;
                if (valid) {
                    const int r = upper_run(rp, tiles, p);
                    const int2 e = sc.sdat[rs[r] + (p - rp[r])];
                    g = e.x;
                    v = e.y;
                }
                int loc = list ? (valid ? sc.lidx[g] : 0) : g - g0;
                if (valid && (loc < 0 || loc >= nk)) {  // impossible for a well-formed plan
                    atomicOr(sc.fault, FAULT_STATIC_KEYS);
                    loc = 0;
                    valid = false;
                }
                int rank = 0;
                uint64_t active = ballot(valid);
                while (active) {
                    const int leader = __ffsll((unsigned long long)active) - 1;
                    const int kl = __shfl(loc, leader, 64);
                    const bool mine = valid && loc == kl;
                    const uint64_t m = ballot(mine);
                    const int c = ctr[kl];
                    if (mine) rank = c + __popcll(m & lanemask_lt());
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    if (lane == leader) ctr[kl] = c + __popcll(m);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    active &= ~m;
                }
                if (valid) {
                    const int32_t kg = sc.lpre[g + 1] - sc.lpre[g];
                    const int32_t need = kg < W ? kg : W;
                    if (rank >= kg - need) {
                        const uint32_t slot =
                            ((uint32_t)sc.pold[g] + (uint32_t)rank) % (uint32_t)W;
                        int32_t *cell = st.ring + (int64_t)g * W + slot;
                        const int32_t old = kg >= W ? 0 : *cell;
                        *cell = v;
                        atomicAdd(reinterpret_cast<unsigned long long *>(&acc[loc]),
                                  (unsigned long long)((long long)v - (long long)old));
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int i = lane; i < nk; i += 64) {
                const int32_t g = list ? list[i] : g0 + i;
                const int32_t kg = sc.lpre[g + 1] - sc.lpre[g];
                if (kg > 0) {
                    const int64_t s = (kg >= W ? 0 : st.sum[g]) + acc[i];
                    st.sum[g] = s;
                    if (out.n_touched) emit_one(out, sc.tidx[g], g, s, sc.ncnt[g]);
                }
            }
        }
    }
    // one record per workgroup: its last worker's end and all its tuples
    if (lane == 0) {
        tend[wv] = (long long)wall_clock64();
        tsum[wv] = tuples;
    }
    __syncthreads();
    if (threadIdx.x == 0 && sc.trace) {
        long long e = 0, s = 0;
        for (int i = 0; i < STATIC_WORKERS_PER_WG; ++i) {
            e = tend[i] > e ? tend[i] : e;
            s += tsum[i];
        }
        const uint32_t hwid = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4);
        const uint32_t xcc = __builtin_amdgcn_s_getreg((15 << 11) | (0 << 6) | 20);
        int64_t *r = sc.trace + 6 * (int64_t)blockIdx.x;
        r[0] = hwid;
        r[1] = xcc;
        r[2] = (int64_t)t0;
        r[3] = e;
        r[4] = s;
        r[5] = STATIC_WORKERS_PER_WG;
    }
}

// ---------------------------------------------- touched list (multi-sub) --
__global__ __launch_bounds__(PLAN_THREADS) void k_touch_reduce(int64_t G, int32_t seq,
                                                               Scratch sc) {
    if (sc.seqp) seq = *sc.seqp;  // captured for replay: the argument would be stale
    __shared__ int red[PLAN_THREADS / 64];
    const int64_t g0 = (int64_t)blockIdx.x * PLAN_CHUNK + (int64_t)threadIdx.x * PLAN_KPT;
    int f[1] = {0}, t[1];
    for (int i = 0; i < PLAN_KPT; ++i)
        if (g0 + i < G && sc.stamp[g0 + i] == seq) ++f[0];
    block_excl_scan<1>(f, t, red);
    if (threadIdx.x == 0) sc.partials[blockIdx.x] = t[0];
}

__global__ __launch_bounds__(PLAN_THREADS) void k_touch_scan(int32_t nblk, Scratch sc) {
    __shared__ int red[PLAN_THREADS / 64];
    const int per = (nblk + PLAN_THREADS - 1) / PLAN_THREADS;
    const int b0 = min(nblk, (int)threadIdx.x * per), b1 = min(nblk, b0 + per);
    int f[1] = {0}, t[1];
    for (int b = b0; b < b1; ++b) f[0] += sc.partials[b];
    block_excl_scan<1>(f, t, red);
    for (int b = b0; b < b1; ++b) {
        const int x = sc.partials[b];
        sc.partials[b] = f[0];
        f[0] += x;
    }
    if (threadIdx.x == 0) sc.tot->n_touched = t[0];
}

__global__ __launch_bounds__(PLAN_THREADS) void k_touch_write(int64_t G, int32_t seq,
                                                              Scratch sc) {
    if (sc.seqp) seq = *sc.seqp;  // captured for replay: the argument would be stale
    __shared__ int red[PLAN_THREADS / 64];
    const int64_t g0 = (int64_t)blockIdx.x * PLAN_CHUNK + (int64_t)threadIdx.x * PLAN_KPT;
    int f[1] = {0}, t[1];
    for (int i = 0; i < PLAN_KPT; ++i)
        if (g0 + i < G && sc.stamp[g0 + i] == seq) ++f[0];
    block_excl_scan<1>(f, t, red);
    int j = f[0] + sc.partials[blockIdx.x];
    for (int i = 0; i < PLAN_KPT; ++i)
        if (g0 + i < G && sc.stamp[g0 + i] == seq) sc.touched[j++] = (int32_t)(g0 + i);
}

// --------------------------------------------------------------- k_emit --
// Results of the most recent batch from the state, in touched-list order.
__global__ __launch_bounds__(EMIT_THREADS) void k_emit(State st, Scratch sc, Out out) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t status = sc.tot->status;
    if (status) {
        if (gid == 0) *out.n_touched = status;
        return;
    }
    const int32_t nt = sc.tot->n_touched;
    if (gid == 0) *out.n_touched = nt;
    for (int64_t j = gid; j < nt; j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = sc.touched[j];
        emit_one(out, (int32_t)j, g, st.sum[g], st.cnt[g]);
    }
}

__global__ void k_reset_totals(Scratch sc) {
    PlanTotals t = {0, 0, 0, 0, 0, 0, 0, 0};
    *sc.tot = t;
}

// ======================================================= several batches --
// Up to SB_K consecutive batches of one query share six launches:
//
//   k_sb_hist   every batch's key histogram (the tiles of all batches).
//   k_sb_sums, k_sb_plan
//               every batch's own balanced plan (buckets, output positions),
//               and the places of the survivors: a tuple can be in a window
//               emitted for its own batch or a later one only if it is
//               among its group's last W tuples of its batch (a tuple that
//               is not is more than W places from the end of every later
//               batch too), so each group's survivors of every batch get
//               consecutive places, batch by batch, in arrival order.
//   k_sb_pass   every tile of every batch reordered by its batch's plan.
//   k_sb_prep   per (batch, bucket): each tuple's rank inside its group,
//               survivors written to their places.
//   k_sb_apply  per group (one wave each; a workgroup for a group with
//               more than APPLY_BUDGET values to read): with C the group's
//               tuples in batches 0..b of the call and S = its window
//               before the call (W values, oldest first; never-written
//               slots hold 0) followed by its new tuples in arrival order,
//               batch b's window is S[C, C + W): its new part is the last
//               min(W, C) survivors up to the end of batch b's, consecutive
//               places; its old part (C < W) is the window sum before the
//               call minus S[0, C).  The final window goes to the ring
//               (Section 3.2: slot nextPos).

// Batch of tile t, given the tiles before each batch (K batches).
__device__ __forceinline__ int sb_batch_of(const int32_t *tile0, int K, int t) {
    int b = 0;
    while (b + 1 < K && tile0[b + 1] <= t) ++b;
    return b;
}

// One histogram tile of one batch per block: its SBH_TILE keys (a thread's
// in chunks of SBH_CHUNK, each chunk's loads in flight together, so that
// registers allow three blocks per CU) counted in LDS as pairs of 16-bit
// counters, group 2i in the low half of word i and 2i + 1 in the high half
// (a tile's count of a group fits 16 bits, so a half never carries into the
// other), the previous call's two most frequent groups in registers; the
// words are the per-tile table's entries as they stand.
__global__ __launch_bounds__(SBH_THREADS) void k_sb_hist(Scratch base, SbBufs sb,
                                                         SbBatches in, int32_t G,
                                                         int32_t seq) {
    constexpr int SBH_CHUNK = 32;
    static_assert(SBH_KPT % SBH_CHUNK == 0 && SBH_CHUNK % 4 == 0, "keys loaded four at a time");
    extern __shared__ uint32_t cpair[];
    const int t = (int)blockIdx.x, tid = (int)threadIdx.x;
    const int b = sb_batch_of(in.htile0, in.K, t);
    const int tile = t - in.htile0[b];
    const int32_t *keys = in.keys[b];
    const int64_t n = in.n[b];
    const bool vec = (in.vec >> b) & 1u;
    const int words = (G + 1) / 2;
    phase_mark(base, PHASE_HIST_PLAN, 0);
    const int32_t hot0 = base.hot[0], hot1 = base.hot[1];
    for (int i = tid; i < words; i += SBH_THREADS) cpair[i] = 0;
    int bad = 0, c0 = 0, c1 = 0;
    for (int ch = 0; ch < SBH_KPT / SBH_CHUNK; ++ch) {
        const int64_t i0 = (int64_t)tile * SBH_TILE + (int64_t)ch * SBH_THREADS * SBH_CHUNK;
        int32_t v[SBH_CHUNK];
#pragma unroll
        for (int j = 0; j < SBH_CHUNK / 4; ++j) {
            const int64_t i = i0 + 4 * ((int64_t)j * SBH_THREADS + tid);
            if (vec && i + 3 < n) {
                // (a streaming load: the reorder then finds fewer of the keys
                // in cache, but the two launches together take less time)
                typedef int v4i __attribute__((ext_vector_type(4)));
                const v4i x = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(keys + i));
                v[4 * j] = x.x; v[4 * j + 1] = x.y; v[4 * j + 2] = x.z; v[4 * j + 3] = x.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[4 * j + e] = (i + e < n) ? keys[i + e] : 0;
            }
        }
        if (base.kmod) {
#pragma unroll
            for (int j = 0; j < SBH_CHUNK; ++j) v[j] = view_key(v[j], base.kmod, G);
        }
        if (ch == 0) __syncthreads();  // (the counters are cleared)
#pragma unroll
        for (int j = 0; j < SBH_CHUNK / 4; ++j) {
            const int64_t i = i0 + 4 * ((int64_t)j * SBH_THREADS + tid);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (i + e >= n) continue;
                const int32_t key = v[4 * j + e];
                if (key < 0 || key >= G) bad = 1;
                else if (key == hot0) ++c0;
                else if (key == hot1) ++c1;
                else atomicAdd(&cpair[key >> 1], 1u << ((key & 1) << 4));
            }
        }
    }
    c0 = wave_total(wave_incl_add(c0));
    c1 = wave_total(wave_incl_add(c1));
    if (lane_id() == 0) {
        if (c0) atomicAdd(&cpair[hot0 >> 1], (uint32_t)c0 << ((hot0 & 1) << 4));
        if (c1) atomicAdd(&cpair[hot1 >> 1], (uint32_t)c1 << ((hot1 & 1) << 4));
    }
    if (__syncthreads_or(bad)) {
        if (tid == 0) atomicExch(sb.sbad + b, seq);
    }
    phase_mark(base, PHASE_HIST_PLAN, 1);
    uint32_t *dense = sb.kt + ((int64_t)b * SBH_TILES + tile) * words;
    for (int i = tid; i < words; i += SBH_THREADS) dense[i] = cpair[i];
    phase_mark(base, PHASE_HIST_PLAN, 2);
}

// The plan of every batch and the survivors' places, one group per thread.
// Every block sums the fields of all groups itself (those before its first
// group give its carries, all of them the totals), so no block waits on
// another.  Fields per batch: light tuples, and heavy groups | touched
// groups << 12; then survivors per group, and 1 for a group whose
// survivors plus old values read exceed APPLY_BUDGET.
static_assert(SUB / SB_HEAVY_MIN < (1 << 12) && (int64_t)PASS_LOCAL_G << 12 < (1LL << 31),
              "heavy groups of a batch fit 12 bits, touched groups the rest of an int");

struct SbGroup {
    int32_t k[SB_K];  // tuples per batch (0 for a rejected batch)
    int32_t cnt0;     // window count before the call
};

__device__ __forceinline__ void sb_fields(const SbGroup &q, int K, int32_t W, int (&x)[SBP_F],
                                          int32_t &kg) {
    int m = 0;
    kg = 0;
#pragma unroll
    for (int b = 0; b < SB_K; ++b) {
        const int32_t k = b < K ? q.k[b] : 0;
        const bool heavy = k >= SB_HEAVY_MIN;
        x[2 * b] = (k > 0 && !heavy) ? k : 0;
        x[2 * b + 1] = (heavy ? 1 : 0) | (k > 0 ? 1 << 12 : 0);
        m += min(k, W);
        kg += k;
    }
    const int lold = (kg > 0 && q.cnt0 > 0) ? min(W, kg) : 0;
    x[2 * SB_K] = m;
    x[2 * SB_K + 1] = m + lold > APPLY_BUDGET ? 1 : 0;
}

// U groups' counters and window counts: every load issued before any is
// used (indexes clamped; groups at or past `end` count nothing).
template <int U>
__device__ __forceinline__ void sb_load_groups(const SbBufs &sb, const State &st,
                                               const bool (&valid)[SB_K], int K, int h0,
                                               int stride, int end, SbGroup (&q)[U]) {
    static_assert(SB_K % 4 == 0, "a group's counters load as int4s");
    constexpr int Q = SB_K / 4;
    int4 ka[U][Q];
    int32_t cn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int h = min(h0 + u * stride, (int)st.G - 1);
        const int4 *p = reinterpret_cast<const int4 *>(sb.kh + (int64_t)h * SB_K);
#pragma unroll
        for (int j = 0; j < Q; ++j) ka[u][j] = p[j];
        cn[u] = st.cnt[h];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int j = 0; j < Q; ++j) keep(ka[u][j]);
        keep(cn[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool in = h0 + u * stride < end;
        int32_t v[SB_K];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            v[4 * j] = ka[u][j].x;
            v[4 * j + 1] = ka[u][j].y;
            v[4 * j + 2] = ka[u][j].z;
            v[4 * j + 3] = ka[u][j].w;
        }
#pragma unroll
        for (int b = 0; b < SB_K; ++b) q[u].k[b] = (in && b < K && valid[b]) ? v[b] : 0;
        q[u].cnt0 = in ? cn[u] : 0;
    }
}

// Plan, first launch: per block of SBS_GROUPS groups, every group's count per
// batch (its histogram tiles summed: thread (pair, batch) sums the tiles of
// two groups of one batch, all its loads in flight together), stored for
// the later steps; then the block's sums of the fields over its groups and
// its two most frequent groups (wave 0, one group per lane).
__global__ __launch_bounds__(SBS_THREADS) void k_sb_sums(State st, Scratch base, SbBufs sb,
                                                         SbBatches in, int32_t seq) {
    static_assert(SBS_GROUPS == 64 && SBS_THREADS == SB_K * SBS_GROUPS / 2,
                  "a thread per (pair of groups, batch); a lane per group after");
    __shared__ int32_t kc[SB_K][SBS_GROUPS];
    const int tid = threadIdx.x, lane = lane_id();
    const int K = in.K;
    const int G = (int)st.G;
    const int32_t W = st.W;
    const int g0 = (int)blockIdx.x * SBS_GROUPS;
    phase_mark(base, PHASE_HIST_PLAN, 3);
    // (each lane's group's window count, for the fields after the barrier,
    // loaded now beside the tile counts)
    const int32_t cnt0 = g0 + lane < G ? st.cnt[g0 + lane] : 0;
    {
        const int pair = tid % (SBS_GROUPS / 2), b = tid / (SBS_GROUPS / 2);
        int nt = 0;
#pragma unroll
        for (int bb = 0; bb < SB_K; ++bb)
            if (b == bb && bb < K) nt = in.htile0[bb + 1] - in.htile0[bb];
        const int64_t row = (G + 1) / 2;
        const int64_t wi = min((int64_t)g0 / 2 + pair, row - 1);
        const uint32_t *p = sb.kt + (int64_t)b * SBH_TILES * row + wi;
        uint32_t w[SBH_TILES];
#pragma unroll
        for (int t = 0; t < SBH_TILES; ++t) w[t] = p[(int64_t)min(t, max(nt - 1, 0)) * row];
        int32_t lo = 0, hi = 0;
#pragma unroll
        for (int t = 0; t < SBH_TILES; ++t)
            if (t < nt) {
                lo += (int32_t)(w[t] & 0xffffu);
                hi += (int32_t)(w[t] >> 16);
            }
        kc[b][2 * pair] = lo;
        kc[b][2 * pair + 1] = hi;
        // A heavy group's tuples in a histogram tile followed by at least W
        // of its tuples in later tiles of the batch cannot be in any window
        // (each has W later tuples of its own batch): the number of such
        // leading tiles, for the reorder to drop them.
        int32_t plo = 0, phi = 0, clo = 0, chi = 0;
#pragma unroll
        for (int t = 0; t < SBH_TILES; ++t)
            if (t < nt) {
                plo += (int32_t)(w[t] & 0xffffu);
                phi += (int32_t)(w[t] >> 16);
                clo += lo - plo >= W ? 1 : 0;
                chi += hi - phi >= W ? 1 : 0;
            }
        const int64_t gl = min((int64_t)g0 + 2 * pair, (int64_t)G - 1);
        if (g0 + 2 * pair < G)
            sb.cut[gl * SB_K + b] = (uint8_t)(lo >= SB_HEAVY_MIN ? clo : 0);
        if (g0 + 2 * pair + 1 < G)
            sb.cut[(gl + 1) * SB_K + b] = (uint8_t)(hi >= SB_HEAVY_MIN ? chi : 0);
    }
    __syncthreads();
    // four waves, a lane per group: every wave forms the fields, wave w
    // sums those with f mod 4 = w; wave 0 stores the counts, wave 1 keeps
    // the two most frequent groups
    constexpr int FW = 4;
    static_assert(FW * 64 <= SBS_THREADS, "the block has four waves");
    const int wv = tid >> 6;
    if (wv >= FW) return;
    const int g = g0 + lane;
    bool valid[SB_K];
#pragma unroll
    for (int b = 0; b < SB_K; ++b) valid[b] = b < K && sb.sbad[b] != seq;
    SbGroup own;
#pragma unroll
    for (int b = 0; b < SB_K; ++b) own.k[b] = (g < G && valid[b]) ? kc[b][lane] : 0;
    own.cnt0 = cnt0;
    if (wv == 0 && g < G) {
        int4 *kp = reinterpret_cast<int4 *>(sb.kh + (int64_t)g * SB_K);
#pragma unroll
        for (int j = 0; j < SB_K / 4; ++j)
            kp[j] = make_int4(kc[4 * j][lane], kc[4 * j + 1][lane], kc[4 * j + 2][lane],
                              kc[4 * j + 3][lane]);
    }
    int x[SBP_F];
    int32_t kg;
    sb_fields(own, K, W, x, kg);
    int32_t *part = sb.part + (int64_t)blockIdx.x * SBP_PART;
#pragma unroll
    for (int f = 0; f < SBP_F; ++f) {
        if (f % FW != wv) continue;
        const int t = wave_total(wave_incl_add(x[f]));
        if (lane == 0) part[f] = t;
    }
    if (wv == 1) {
        Top2 top;
        if (kg > 0) top.add(((unsigned long long)(uint32_t)kg << 32) | (uint32_t)g);
        top2_wave(top);
        if (lane == 0) {
            reinterpret_cast<unsigned long long *>(part + SBP_F)[0] = top.a;
            reinterpret_cast<unsigned long long *>(part + SBP_F)[1] = top.b;
        }
    }
    phase_mark(base, PHASE_HIST_PLAN, 4);
}

// Plan, second launch: every batch's own balanced plan and the survivors'
// places, one group per thread, from the blocks' sums (those of the blocks
// before this one give its carries, all of them the totals).  The batches
// are split over PLAN_SPLIT rows of blocks (blockIdx.y): row Q takes
// batches [Q * PLAN_KQ, (Q + 1) * PLAN_KQ) and so scans only their fields
// and the two per group; row 0 also writes the per-group places.
constexpr int PLAN_SPLIT = 5;
constexpr int PLAN_KQ = SB_K / PLAN_SPLIT;
constexpr int PLAN_NF = 2 * PLAN_KQ + 2;
static_assert(SB_K % PLAN_SPLIT == 0, "the plan's rows take equal shares of the batches");

// LDS of a plan block (row-local field i: batch fields 2 b0 + i, then the
// survivors and big-group fields).
struct PlanLds {
    int wown[SBP_THREADS / 64][PLAN_NF];
    int wbase[SBP_THREADS / 64][PLAN_NF];  // exclusive field values at each wave's first group
    int ftot[PLAN_NF];                     // field totals over all groups
    int bpre[PLAN_NF];                     // field sums of the blocks before this one
    __align__(8) int32_t parts[SBS_BLOCKS_MAX * SBP_PART];  // every sums block's
};

template <int Q>
__device__ __forceinline__ void sb_plan_row(const State &st, const Scratch &base,
                                            const SbBufs &sb, const SbBatches &in, int32_t seq,
                                            PlanLds &L) {
    constexpr int NW = SBP_THREADS / 64;
    constexpr int B0 = Q * PLAN_KQ;
    // the global field of row-local field i
    auto gf = [](int i) { return i < 2 * PLAN_KQ ? 2 * B0 + i : 2 * SB_K + (i - 2 * PLAN_KQ); };
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int K = in.K;
    if (Q > 0 && B0 >= K) return;  // (no batch of this row in the call)
    const int G = (int)st.G;
    const int32_t W = st.W;
    const int nblk = (G + SBS_GROUPS - 1) / SBS_GROUPS;  // sums blocks
    const int kfirst = (int)blockIdx.x * (SBP_THREADS / SBS_GROUPS);  // this block's first
    const int gb = (int)blockIdx.x * SBP_THREADS, g = gb + tid;
    bool valid[SB_K];
#pragma unroll
    for (int b = 0; b < SB_K; ++b) valid[b] = b < K && sb.sbad[b] != seq;
    SbGroup own[1];
    sb_load_groups<1>(sb, st, valid, K, g, 0, G, own);
    // a heavy item's dropped tiles per batch of the row (a group's SB_K
    // bytes together), loaded here with the rest rather than in the loop
    static_assert(SB_K % 4 == 0, "a group's dropped-tile counts load as words");
    uint32_t cutw[SB_K / 4];
    {
        const uint32_t *cp =
            reinterpret_cast<const uint32_t *>(sb.cut + (int64_t)min(g, G - 1) * SB_K);
#pragma unroll
        for (int j = 0; j < SB_K / 4; ++j)
            if (4 * j + 3 >= B0 && 4 * j < B0 + PLAN_KQ) cutw[j] = cp[j];
    }
    {  // every block's partials, loaded together
        constexpr int PER = (SBS_BLOCKS_MAX * SBP_PART + SBP_THREADS - 1) / SBP_THREADS;
        const int np = nblk * SBP_PART;
        int32_t v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) v[j] = sb.part[min(tid + j * SBP_THREADS, np - 1)];
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (tid + j * SBP_THREADS < np) L.parts[tid + j * SBP_THREADS] = v[j];
    }
    __syncthreads();
    // row field i summed over the sums blocks before this block and over
    // all, by wave i mod NW, its lanes striding over the blocks
#pragma unroll
    for (int i = 0; i < PLAN_NF; ++i) {
        if (i % NW != wv) continue;
        int p = 0, t = 0;
#pragma unroll
        for (int j = 0; j < SBS_BLOCKS_MAX / 64; ++j) {
            const int k = lane + 64 * j;
            const int v = k < nblk ? L.parts[k * SBP_PART + gf(i)] : 0;
            p += k < kfirst ? v : 0;
            t += v;
        }
        p = wave_total(wave_incl_add(p));
        t = wave_total(wave_incl_add(t));
        if (lane == 0) {
            L.bpre[i] = p;
            L.ftot[i] = t;
        }
    }
    int wex[PLAN_NF];
    int32_t own_big;
    {
        int x[SBP_F];
        int32_t kg;
        sb_fields(own[0], K, W, x, kg);
#pragma unroll
        for (int i = 0; i < PLAN_NF; ++i) {
            const int incl = wave_incl_add(x[gf(i)]);
            if (lane == 63) L.wown[wv][i] = incl;
            wex[i] = incl - x[gf(i)];
        }
        own_big = x[2 * SB_K + 1];
    }
    __syncthreads();
    if (tid < PLAN_NF) {  // thread i: field i's value at each wave's start
        const int i = tid;
        int run = L.bpre[i];
        for (int w = 0; w < NW; ++w) {
            L.wbase[w][i] = run;
            run += L.wown[w][i];
        }
    }
    __syncthreads();
    // (by row-local field)
    auto ex = [&](int i) { return L.wbase[wv][i] + wex[i]; };
    auto tot = [&](int i) { return L.ftot[i]; };
    constexpr int FS = 2 * PLAN_KQ, FB = 2 * PLAN_KQ + 1;  // survivors, big groups
    phase_mark(base, PHASE_HIST_PLAN, 6);
    if (g < G) {
        int m_before = 0;  // survivors of this group in the batches before b
#pragma unroll
        for (int b = 0; b < B0; ++b) m_before += min(own[0].k[b], W);
#pragma unroll
        for (int bl = 0; bl < PLAN_KQ; ++bl) {
            const int b = B0 + bl;
            if (b >= K || !valid[b]) continue;
            const Scratch sc = sb_set(sb, base, b, G);
            const int32_t k = own[0].k[b];
            const int exl = ex(2 * bl), exh = ex(2 * bl + 1) & 0xfff,
                      ext = ex(2 * bl + 1) >> 12;
            const int32_t nl = (tot(2 * bl) + SB_LIGHT_BUDGET - 1) / SB_LIGHT_BUDGET;
            sc.lpre[g] = exl;
            sb.so[(int64_t)b * G + g] = ex(FS) + m_before;
            if (k > 0) {
                sc.tidx[g] = ext;
                if (k >= SB_HEAVY_MIN) {
                    sc.bucket[g] =
                        (nl + exh) | (int32_t)(((cutw[b / 4] >> (8 * (b % 4))) & 0xffu) << 16);
                    if ((uint32_t)exh < (uint32_t)SB_NB_MAX) sc.hkey[exh] = g;
                } else {
                    sc.bucket[g] = (exl + k - 1) / SB_LIGHT_BUDGET;
                    const int32_t m = (exl + SB_LIGHT_BUDGET - 1) / SB_LIGHT_BUDGET;
                    if ((int64_t)m * SB_LIGHT_BUDGET <= (int64_t)exl + k - 1 &&
                        (uint32_t)m < (uint32_t)SB_NB_MAX)
                        sc.bstart[m] = g;
                }
                // the last batch's touched list serves cq_results after the call
                if (b == K - 1) base.touched[ext] = g;
            }
            m_before += min(k, W);
        }
        if (Q == 0) {
            sb.gsb[g] = ex(FS);
            sb.gbig[g] = own_big;
            if (own_big) sb.big[ex(FB)] = g;
        }
    }
    // batch b's totals by thread 0 of block b mod grid of its row, so that
    // no block writes many (an unrolled loop: the batches' arguments are
    // indexed by constants)
    const int grid = (int)gridDim.x;
#pragma unroll
    for (int bl = 0; bl < PLAN_KQ; ++bl) {
        const int b = B0 + bl;
        if (tid != 0 || b >= K || b % grid != (int)blockIdx.x) continue;
        const Scratch sc = sb_set(sb, base, b, G);
        PlanTotals t;
        const int32_t nl = (tot(2 * bl) + SB_LIGHT_BUDGET - 1) / SB_LIGHT_BUDGET;
        t.n_light_buckets = valid[b] ? nl : 0;
        t.n_heavy = valid[b] ? tot(2 * bl + 1) & 0xfff : 0;
        t.light_tuples = valid[b] ? tot(2 * bl) : 0;
        t.n_touched = valid[b] ? tot(2 * bl + 1) >> 12 : 0;
        t.status = valid[b] ? 0 : CQ_ERR_KEY_RANGE;
        t.n_buckets = t.n_light_buckets + t.n_heavy;
        t.tiles = (int32_t)((in.n[b] + PASS_TILE - 1) / PASS_TILE);
        t.sub_touched = t.n_touched;
        *sc.tot = t;
        if (valid[b]) {
            sc.lpre[G] = t.light_tuples;
            sc.bstart[nl] = G;
        }
        if (in.out[b].n_touched) *in.out[b].n_touched = t.status ? t.status : t.n_touched;
        if (b == K - 1) *base.tot = t;
        if (t.n_buckets > SB_NB_MAX) atomicOr(base.fault, FAULT_BUCKETS);
    }
    if (Q == 0) {
        if (blockIdx.x == 0 && tid == 64) {
            sb.gsb[G] = tot(FS);
            sb.ntot[0] = tot(FB);
            sb.ntot[1] = tot(FS);
        }
        // the call's two most frequent groups, for the next histogram, by the
        // last wave of the last block
        if (blockIdx.x == gridDim.x - 1 && wv == NW - 1) {
            Top2 top;
#pragma unroll
            for (int j = 0; j < SBS_BLOCKS_MAX / 64; ++j) {
                const int k = lane + 64 * j;
                if (k < nblk) {
                    const unsigned long long *p = reinterpret_cast<const unsigned long long *>(
                        L.parts + k * SBP_PART + SBP_F);
                    top.add(p[0]);
                    top.add(p[1]);
                }
            }
            top2_wave(top);
            if (lane == 0) {
                base.hot[0] = top.a ? (int32_t)(uint32_t)top.a : -1;
                base.hot[1] = top.b ? (int32_t)(uint32_t)top.b : -1;
            }
        }
    }
}

// Row y's plan (the row index a template argument, so that its batches'
// fields are indexed by constants).
template <int Q>
__device__ __forceinline__ void sb_plan_rows(int y, const State &st, const Scratch &base,
                                             const SbBufs &sb, const SbBatches &in, int32_t seq,
                                             PlanLds &L) {
    if (y == Q)
        sb_plan_row<Q>(st, base, sb, in, seq, L);
    else if constexpr (Q + 1 < PLAN_SPLIT)
        sb_plan_rows<Q + 1>(y, st, base, sb, in, seq, L);
}

__global__ __launch_bounds__(SBP_THREADS) void k_sb_plan(State st, Scratch base, SbBufs sb,
                                                         SbBatches in, int32_t seq) {
    __shared__ PlanLds L;
    phase_mark(base, PHASE_HIST_PLAN, 5);
    sb_plan_rows<0>((int)blockIdx.y, st, base, sb, in, seq, L);
    phase_mark(base, PHASE_HIST_PLAN, 7);
}

// The reorder of every tile of every batch: one workgroup per CU works
// through a contiguous run of tiles, two tiles ahead: while tile t is
// reordered in LDS, the keys and values of tile t + 2 are on their way and
// the buckets of tile t + 1 are being gathered, so each tile waits only on
// its own LDS work.
// A reorder workgroup's tiles: batch, tile index inside it, the batch's
// tuples (looked up once, not per prefetch; the arrays come from the kernel
// argument, so that their loads stay global rather than generic ones).
struct SbTile {
    int32_t n, b, tile;
};
constexpr int SB_PASS_PER = (SB_K * PASS_TILES_MAX + SB_PASS_GRID - 1) / SB_PASS_GRID;  // tiles per reorder workgroup at most
static_assert(SB_K * PASS_TILES_MAX <= SB_PASS_PER * SB_PASS_GRID,
              "every workgroup's tiles fit its table");

// LDS of a reorder workgroup (bytes): per-wave counters, then the reordered
// tile, whose bytes hold the per-wave leader tables until the ranks are done
constexpr int SBL_LEAD = 2048;                                  // leader bytes per wave
constexpr int SBL_WC = 0;                                       // u16[PASS_WAVES][SB_NB_MAX]
constexpr int SBL_STAGE = (SBL_WC + 2 * PASS_WAVES * SB_NB_MAX + 15) & ~15;  // int2[PASS_TILE]
constexpr int SBL_BYTES = SBL_STAGE + 8 * PASS_TILE;
static_assert(SB_NB_MAX - 2 <= SBL_LEAD, "a leader entry for every bucket id");
static_assert(PASS_WAVES * SBL_LEAD <= 8 * PASS_TILE, "leader tables fit the tile's bytes");

// (registers for four waves per SIMD: two workgroups per CU)
__global__ __launch_bounds__(PASS_THREADS, 4) void k_sb_pass(State st, Scratch base, SbBufs sb,
                                                             SbBatches in, int32_t seq) {
    __shared__ __align__(16) char pool[SBL_BYTES];
    __shared__ int32_t ts[SB_NB_MAX + 1];
    __shared__ int red[PASS_WAVES];
    __shared__ SbTile tl[SB_PASS_PER];
    constexpr int R = PASS_ROUNDS;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int K = in.K;
    const int64_t G = st.G;
    const int T = in.ptile0[K];
    const int per = (T + (int)gridDim.x - 1) / (int)gridDim.x;
    const int t_begin = (int)blockIdx.x * per, t_end = min(T, t_begin + per);
    if (t_begin >= t_end) return;
    if (tid < t_end - t_begin) {
        const int t = t_begin + tid;
        SbTile x = {0, 0, 0};
#pragma unroll
        for (int b = 0; b < SB_K; ++b)
            if (b < K && in.ptile0[b] <= t && t < in.ptile0[b + 1])
                x = {(int32_t)in.n[b], b, t - in.ptile0[b]};
        tl[tid] = x;
    }
    __syncthreads();
    // position of this thread's round r inside a tile
    auto pos = [&](int r) { return wave * (PASS_TILE / PASS_WAVES) + r * 64 + lane; };
    auto load_kv = [&](const SbTile &x, int32_t (&k)[R], int32_t (&v)[R]) {
        const int32_t tb = x.tile * PASS_TILE, last = x.n - 1;
        const int32_t *kp = in.keys[x.b], *vp = in.values[x.b];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t i = (uint32_t)min(tb + pos(r), last);
            // (streaming loads: the batch is read once here and not again)
            k[r] = __builtin_nontemporal_load(kp + i);
            v[r] = __builtin_nontemporal_load(vp + i);
        }
    };
    // a tile's group views and buckets: loads issued here and first used in
    // the next iteration (positions past the batch are masked there), so
    // that they stay in flight meanwhile
    auto gather = [&](const SbTile &x, int32_t (&k)[R], int32_t (&bk)[R]) {
        const int32_t *bucket = sb.bucket + (int64_t)x.b * G;
        if (base.kmod) {  // (a uniform branch: the reduction costs nothing when off)
#pragma unroll
            for (int r = 0; r < R; ++r) k[r] = view_key(k[r], base.kmod, G);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // (a rejected batch's keys may be out of range: clamped, unused)
            const uint32_t kc = (uint32_t)k[r] < (uint32_t)G ? (uint32_t)k[r] : 0u;
            bk[r] = bucket[kc];
        }
    };
    // (the table's entries are the same in every lane: taken as scalars, so
    // that loads address them as a scalar base plus a 32-bit offset)
    auto tile_of = [&](int t) {
        const SbTile &e = tl[min(t, t_end - 1) - t_begin];
        SbTile x;
        x.n = __builtin_amdgcn_readfirstlane(e.n);
        x.b = __builtin_amdgcn_readfirstlane(e.b);
        x.tile = __builtin_amdgcn_readfirstlane(e.tile);
        return x;
    };
    int32_t kA[R], vA[R], bA[R], kB[R], vB[R], bB[R], kC[R], vC[R], lr[R];
    // Tile t's keys, values, buckets and plan totals are in registers when
    // its iteration starts.  During it, tile t + 2's keys and values and tile
    // t + 1's buckets and totals are loaded; they are waited for only after
    // tile t's LDS work and before its stores, so that no wait at the top of
    // an iteration has stores or younger loads in front of it.  (Past the
    // run the last tile is loaded again and not used: every load stays
    // unconditional.)
    {
        const SbTile x0 = tile_of(t_begin);
        load_kv(x0, kA, vA);
        load_kv(tile_of(t_begin + 1), kB, vB);
        gather(x0, kA, bA);
    }
    PlanTotals tA = sb.tot[tile_of(t_begin).b];
    // (waited for here, so that no load of this prologue is still counted
    // where the loop's first tile starts: the top of every iteration then
    // waits on nothing, not even the previous tile's stores)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        keep(kA[r]);
        keep(vA[r]);
        keep(bA[r]);
        keep(kB[r]);
        keep(vB[r]);
    }
    keep(tA.status);
    keep(tA.n_buckets);
    for (int t = t_begin; t < t_end; ++t) {
        phase_mark(base, PHASE_PASS, 0);
        const SbTile x = tile_of(t), x1 = tile_of(t + 1), x2 = tile_of(t + 2);
        load_kv(x2, kC, vC);
        gather(x1, kB, bB);
        PlanTotals tB = sb.tot[x1.b];
        const int b = x.b;
        const int64_t tb = (int64_t)x.tile * PASS_TILE;
        const int tile_n = (int)min((int64_t)PASS_TILE, x.n - tb);
        auto arrive = [&]() {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                keep(kC[r]);
                keep(vC[r]);
                keep(bB[r]);
            }
            keep(tB.status);
            keep(tB.n_buckets);
        };
        const int32_t nA = tA.n_buckets;
        if (!tA.status && nA <= SB_NB_MAX - 2) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // (a heavy group's bucket carries the histogram tiles of
                // the batch whose tuples of it are dropped)
                const int64_t i = tb + pos(r);
                bA[r] = i < x.n && (int32_t)(i / SBH_TILE) >= (bA[r] >> 16) ? (bA[r] & 0xffff)
                                                                          : nA;
                lr[r] = 0;
            }
            const Scratch sc = sb_set(sb, base, b, G);
            pass_split<SB_NB_MAX, SBL_LEAD>(
                kA, vA, bA, lr, nA, tb, tile_n, x.tile, sc,
                reinterpret_cast<uint16_t *>(pool + SBL_WC),
                reinterpret_cast<int2 *>(pool + SBL_STAGE), ts, red,
                reinterpret_cast<uint8_t *>(pool + SBL_STAGE), [] {}, arrive);
        } else {
            if (!tA.status && tid == 0) atomicOr(base.fault, FAULT_BUCKETS);  // (no plan makes
            arrive();                                                          // this many)
        }
        __syncthreads();  // (the next tile reuses the LDS)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            kA[r] = kB[r];
            vA[r] = vB[r];
            bA[r] = bB[r];
            kB[r] = kC[r];
            vB[r] = vC[r];
        }
        tA = tB;
    }
}

// LDS of one survivor wave (bytes): per run of its bucket (one per tile) the
// first bucket position and the staged start; per bucket position its run;
// per group (indexed by its first position in the bucket) a leader byte and
// the tuples ranked so far.
constexpr int SPW_P = 0;                                 // i32[PASS_TILES_MAX + 1]
constexpr int SPW_S = SPW_P + 4 * (PASS_TILES_MAX + 4);  // i32[PASS_TILES_MAX]
constexpr int SPW_RT = SPW_S + 4 * PASS_TILES_MAX;       // u8[SB_LIGHT_CAP]
constexpr int SPW_LEAD = SPW_RT + SB_LIGHT_CAP;          // u8[SB_LIGHT_CAP]
constexpr int SPW_CNT = SPW_LEAD + SB_LIGHT_CAP;         // u16[SB_LIGHT_CAP]
constexpr int SPW_BYTES = SPW_CNT + 2 * SB_LIGHT_CAP;
static_assert(PASS_TILES_MAX == 4 * 64, "four runs per lane");
static_assert(PASS_TILES_MAX <= 256, "run ids fit a byte");
static_assert(SB_LIGHT_CAP % 512 == 0, "light buckets in halves of eight rounds");


// Survivors, one (batch, bucket) item per wave.  A light bucket's tuples
// are read in arrival order (its runs in tile order), ranked inside their
// groups in rounds of 64 (the lanes of a round that share a group elect a
// leader through a byte table, 6 ballots over its lane id, as the reorder
// does), and each group's last min(k, W) written to their places.  A heavy
// bucket holds one group: its last min(k, W) tuples are copied, and their
// sum kept (the group's whole window for that batch when the batch holds at
// least W of its tuples).
__global__ __launch_bounds__(UPD_THREADS) void k_sb_prep(State st, Scratch base, SbBufs sb,
                                                         SbBatches in) {
    constexpr int WPB = UPD_THREADS / 64;
    __shared__ __align__(16) char smem[WPB * SPW_BYTES];
    __shared__ int items0[SB_K + 1];
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int K = in.K;
    const int64_t G = st.G;
    const int32_t W = st.W;
    phase_mark(base, PHASE_SB_PREP, 0);
    if (tid < SB_K) {  // every batch's item count, loaded together
        const PlanTotals t = sb.tot[tid < K ? tid : 0];
        items0[tid + 1] = (tid < K && !t.status) ? t.n_buckets : 0;
    }
    __syncthreads();
    if (tid == 0) {
        items0[0] = 0;
        for (int b = 0; b < SB_K; ++b) items0[b + 1] += items0[b];
    }
    __syncthreads();
    const int items = items0[K];
    char *my = smem + wv * SPW_BYTES;
    int32_t *P = reinterpret_cast<int32_t *>(my + SPW_P);
    int32_t *RS = reinterpret_cast<int32_t *>(my + SPW_S);
    uint8_t *rt = reinterpret_cast<uint8_t *>(my + SPW_RT);
    uint8_t *lead = reinterpret_cast<uint8_t *>(my + SPW_LEAD);
    uint16_t *cnt = reinterpret_cast<uint16_t *>(my + SPW_CNT);
    const int NWV = (int)gridDim.x * WPB;
    phase_mark(base, PHASE_SB_PREP, 1);
    for (int it = (int)blockIdx.x * WPB + wv; it < items; it += NWV) {
        wave_lds_sync();  // (the previous item's reads of the tables are done)
        const int b = sb_batch_of(items0, K, it);
        const Scratch sc = sb_set(sb, base, b, G);
        const int32_t *so = sb.so + (int64_t)b * G;
        const PlanTotals t = *sc.tot;
        const int kk = it - items0[b];
        const int NB = t.n_buckets, nl = t.n_light_buckets;
        const int tiles = (int)((in.n[b] + PASS_TILE - 1) / PASS_TILE);
        const bool light = kk < nl;
        // the bucket's runs, lane l holding tiles 4l .. 4l+3, and its facts,
        // loaded together
        int32_t rs4[4], rl4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int tt = 4 * lane + j, tc = min(tt, tiles - 1);
            const int32_t *row = sc.rowstart + (int64_t)tc * (NB + 1);
            const int32_t r0 = row[kk], r1 = row[kk + 1];
            rs4[j] = tc * PASS_TILE + r0;
            rl4[j] = tt < tiles ? r1 - r0 : 0;
        }
        const int32_t fa = light ? sc.bstart[kk] : sc.hkey[kk - nl];
        const int32_t fz = light ? sc.bstart[kk + 1] : 0;
        int size;
        {
            const int loc = rl4[0] + rl4[1] + rl4[2] + rl4[3];
            const int incl = wave_incl_add(loc);
            size = wave_total(incl);
            int ex = incl - loc;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                P[4 * lane + j] = ex;
                RS[4 * lane + j] = rs4[j];
                ex += rl4[j];
            }
            if (lane == 0) P[PASS_TILES_MAX] = size;
        }
        if (size <= 0) continue;
        if (!light) {
            const int32_t g = fa;
            const int32_t first = size - min(size, W);
            const int32_t base_x = so[g] - first;
            wave_lds_sync();
            constexpr int HU = 8;
            long long acc = 0;
            for (int p0 = first + lane; p0 < size; p0 += HU * 64) {
                int32_t v[HU];
#pragma unroll
                for (int u = 0; u < HU; ++u) {
                    const int p = min(p0 + u * 64, size - 1);
                    const int r = upper_run(P, tiles, p);
                    v[u] = sc.sdat[RS[r] + (p - P[r])].y;
                }
#pragma unroll
                for (int u = 0; u < HU; ++u)
                    if (p0 + u * 64 < size) {
                        sb.xs[base_x + p0 + u * 64] = v[u];
                        acc += v[u];
                    }
            }
            acc = wave_sum_ll(acc);
            if (lane == 0) sb.tb[(int64_t)b * G + g] = acc;
            continue;
        }
        const int32_t a = fa, z = fz;
        const int32_t s0 = sc.lpre[a];
        if (size > SB_LIGHT_CAP || sc.lpre[z] - s0 != size) {  // impossible for a well-formed plan
            if (lane == 0) atomicOr(sc.fault, FAULT_LIGHT_SIZE);
            continue;
        }
        // every position's run: each non-empty run's id at its first
        // position, then a running maximum (run ids grow with position);
        // lane l owns positions 16l .. 16l+15 here
        constexpr int PPL = SB_LIGHT_CAP / 64;
#pragma unroll
        for (int j = 0; j < PPL / 4; ++j)
            reinterpret_cast<uint32_t *>(rt)[lane * (PPL / 4) + j] = 0;
#pragma unroll
        for (int j = 0; j < 2 * SB_LIGHT_CAP / 4 / 64; ++j)
            reinterpret_cast<uint32_t *>(cnt)[lane + 64 * j] = 0;
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (rl4[j] > 0) rt[P[4 * lane + j]] = (uint8_t)(4 * lane + j);
        wave_lds_sync();
        {
            int mloc = 0, loc[PPL];
#pragma unroll
            for (int i = 0; i < PPL; ++i) {
                mloc = max(mloc, (int)rt[PPL * lane + i]);
                loc[i] = mloc;
            }
            const int incl = wave_incl_max(mloc);
            int before = __shfl_up(incl, 1, 64);
            if (lane == 0) before = 0;
            wave_lds_sync();
#pragma unroll
            for (int i = 0; i < PPL; ++i) rt[PPL * lane + i] = (uint8_t)max(before, loc[i]);
        }
        wave_lds_sync();
        // rounds of 64 positions in arrival order, in halves of eight
        for (int h = 0; h < size; h += 512) {
            constexpr int RH = 8;
            int2 e[RH];
#pragma unroll
            for (int r = 0; r < RH; ++r) {
                const int p = min(h + r * 64 + lane, size - 1);
                const int tt = rt[p];
                e[r] = sc.sdat[RS[tt] + (p - P[tt])];
            }
            int32_t l0[RH], l1[RH], dst[RH];
#pragma unroll
            for (int r = 0; r < RH; ++r) {
                const int32_t g = e[r].x;
                const int32_t gc = g >= a && g < z ? g : a;
                l0[r] = sc.lpre[gc];
                l1[r] = sc.lpre[gc + 1];
                dst[r] = so[gc];
            }
#pragma unroll
            for (int r = 0; r < RH; ++r) {
                const int p = h + r * 64 + lane;
                const int32_t g = e[r].x;
                bool valid = p < size && g >= a && g < z && l1[r] > l0[r];
                const int p0 = valid ? l0[r] - s0 : 0;
                if (valid && (p0 < 0 || p0 >= size)) {  // impossible for a well-formed plan
                    atomicOr(sc.fault, FAULT_LIGHT_SIZE);
                    valid = false;
                }
                if (valid)
                    __hip_atomic_store(lead + p0, (uint8_t)lane, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
                wave_lds_sync();
                const int L = valid ? (int)__hip_atomic_load(lead + p0, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_WAVEFRONT)
                                    : 0;
                const uint64_t m = match_lane_id(valid, L);
                if (valid) {
                    const int below = lanes_below(m);
                    const int c = cnt[p0];
                    const int32_t rank = c + below;
                    if (below == 0) cnt[p0] = (uint16_t)(c + __popcll(m));
                    const int32_t k = l1[r] - l0[r];
                    const int32_t first = k - min(k, W);  // rank of the first survivor
                    if (rank >= first) sb.xs[dst[r] + (rank - first)] = e[r].y;
                }
                wave_lds_sync();
            }
        }
    }
    phase_mark(base, PHASE_SB_PREP, 5);
}

// Lanes of a group's facts in the apply step's waves (A: one int per lane,
// lanes [0, SB_K) its tuples per batch; B: one int64 per lane, lanes [0,
// SB_K) a heavy item's survivor sum, lane SB_K the window sum).
constexpr int AF_TIX = SB_K, AF_POS = 2 * SB_K, AF_CNT = 2 * SB_K + 1,
              AF_GS = 2 * SB_K + 2, AF_BIG = 2 * SB_K + 4;
static_assert(AF_BIG < 64 && SB_K <= 32, "a group's facts fit one wave, a batch per lane");

// A 64-bit value of lane l (a wave-uniform lane).
__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Group g's facts for the calling wave's lanes (a group past the last reads
// the last group's).
__device__ __forceinline__ void apply_facts(const State &st, const SbBufs &sb, int K, int g,
                                            int32_t &A, int64_t &B) {
    const int lane = lane_id();
    const int G = (int)st.G;
    g = min(g, G - 1);
    const int b = lane % SB_K;
    const int bb = b < K ? b : 0;
    const int32_t *pa = lane < AF_TIX   ? sb.kh + (int64_t)g * SB_K + b
                        : lane < AF_POS ? sb.tidx + (int64_t)bb * G + g
                        : lane == AF_POS ? st.pos + g
                        : lane == AF_CNT ? st.cnt + g
                        : lane == AF_GS ? sb.gsb + g
                        : lane == AF_GS + 1 ? sb.gsb + g + 1
                                            : sb.gbig + g;
    const int64_t *pb = lane < SB_K ? sb.tb + (int64_t)bb * G + g : st.sum + g;
    A = *global_ptr(pa);
    B = *global_ptr(pb);
}

// A group's facts as the apply step uses them: the wave-uniform ones, and,
// in lane b < SB_K, batch b's: its tuples k, the group's tuples in batches
// 0..b (c), its output position, the places [lo, hi) of the survivors its
// window holds, the old window values it no longer holds (the first cb,
// while fewer than W tuples have arrived in the call), whether its own
// survivors are its whole window (a heavy item whose sum the prep step
// left) and that sum.  Lanes past SB_K and batches not valid have k = 0.
struct ApplyFacts {
    int32_t pos0, cnt0, gs, m, kg, lold;
    int64_t sum0;
    int last;  // the group's last batch in the call
    bool need_x, any_whole;
    int32_t k, c, tix, lo, hi, cb;
    int64_t tb;
    bool whole;
};

__device__ __forceinline__ ApplyFacts apply_unpack(int32_t A, int64_t B, uint32_t vmask,
                                                  int32_t W) {
    const int lane = lane_id();
    ApplyFacts f;
    f.k = (lane < SB_K && ((vmask >> lane) & 1u)) ? A : 0;
    f.c = wave_incl_add(f.k);
    f.kg = __builtin_amdgcn_readlane(f.c, 63);
    const uint64_t nz = ballot(f.k > 0);
    f.last = nz ? 63 - __builtin_clzll(nz) : 0;
    f.tix = __shfl(A, (AF_TIX + lane) & 63, 64);
    f.pos0 = __builtin_amdgcn_readlane(A, AF_POS);
    f.cnt0 = __builtin_amdgcn_readlane(A, AF_CNT);
    f.gs = __builtin_amdgcn_readlane(A, AF_GS);
    f.m = __builtin_amdgcn_readlane(A, AF_GS + 1) - f.gs;
    f.sum0 = readlane64(B, SB_K);
    f.tb = B;
    f.lold = f.cnt0 > 0 ? min(W, f.kg) : 0;
    f.hi = wave_incl_add(min(f.k, W));
    f.lo = f.hi - min(W, f.c);
    f.cb = (f.k > 0 && f.c < W && f.lold) ? f.c : 0;
    f.whole = f.k >= W && f.k >= SB_HEAVY_MIN;
    f.need_x = ballot(f.k > 0 && !f.whole) != 0;
    f.any_whole = ballot(f.whole) != 0;
    return f;
}

// Lane b's result of batch b for group g (s: its window sum), and, by the
// lane of the group's last batch, the group's final state.
__device__ __forceinline__ void apply_emit(const State &st, const Out *outs, int g,
                                           const ApplyFacts &f, long long s) {
    const int b = lane_id();
    if (b >= SB_K || f.k <= 0) return;
    const int32_t W = st.W;
    emit_one(outs[b], f.tix, g, s, (int32_t)min((int64_t)W, (int64_t)f.cnt0 + f.c));
    if (b == f.last) {
        st.sum[g] = s;
        st.pos[g] = (int32_t)(((uint32_t)f.pos0 + (uint32_t)f.kg) % (uint32_t)W);
        st.cnt[g] = (int32_t)min((int64_t)W, (int64_t)f.cnt0 + f.kg);
    }
}

// One wave's pass over elements [e0, e1) of a sequence, 64 a round and
// RU rounds' loads issued before any is used (more rounds in flight for
// longer runs): load(e) reads element e,
// use(e, loaded) does what follows (stores) and gives its value.  Each
// lane's points q[j] inside (e0, e1] get the sum of the elements [e0, q[j])
// in pre[j] (others keep theirs), from the round's inclusive prefix sum at
// q[j] - 1 plus the rounds before; returns the sum of [e0, e1).
template <int RU, int NP, class Load, class Use>
__device__ __forceinline__ long long apply_run(int32_t e0, int32_t e1, const int32_t (&q)[NP],
                                               long long (&pre)[NP], Load &&load, Use &&use) {
    const int lane = lane_id();
    long long carry = 0;
    for (int32_t r0 = e0; r0 < e1; r0 += RU * 64) {
        decltype(load(0)) t[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u)  // (rounds past the run are not loaded)
            if (r0 + u * 64 < e1) t[u] = load(min(r0 + u * 64 + lane, e1 - 1));
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int32_t base = r0 + u * 64;
            if (base >= e1) break;
            const int32_t e = base + lane;
            const long long x = e < e1 ? use(e, t[u]) : 0LL;
            const long long S = wave_incl_add64(x);
            bool here[NP], any = false;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                here[j] = (uint32_t)(q[j] - 1 - base) < 64u && q[j] <= e1;
                any |= here[j];
            }
            if (ballot(any)) {
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    const long long v = __shfl(S, (q[j] - 1 - base) & 63, 64);
                    if (here[j]) pre[j] = carry + v;
                }
            }
            carry += readlane64(S, 63);
        }
    }
    return carry;
}

// Group g by one wave, its facts in A and B (lanes AF_*).  Batch b's
// window sum, in lane b: when every window of the call reaches back before
// it (kg <= W, no batch whole), the sum before the call plus the
// differences (new - old) of the group's tuples x < c_b, tuple x taking
// slot pos0 + x mod W; otherwise the survivors at places [lo_b, hi_b) less
// the old values [0, cb_b), plus the sum before the call while c_b < W.
// Both are prefix sums of one sequence (the differences; the old values
// then the survivors) read at each batch's points.
__device__ void apply_wave(const State &st, const SbBufs &sb, const Out *outs, uint32_t vmask,
                           int g, int32_t A, int64_t B) {
    const int32_t W = st.W;
    const ApplyFacts f = apply_unpack(A, B, vmask, W);
    if (f.kg == 0) return;
    int32_t *ring = st.ring + (int64_t)g * W;
    const int32_t *xs = sb.xs + f.gs;
    const int32_t unread = W - f.cnt0;
    const uint32_t pos0 = (uint32_t)f.pos0;
    if (f.kg <= W && !f.any_whole) {
        const int32_t q[1] = {f.k > 0 ? f.c : 0};
        long long pre[1] = {0};
        apply_run<8>(
            0, f.kg, q, pre,
            [&](int32_t x) {
                uint32_t slot = pos0 + (uint32_t)x;
                slot = slot >= (uint32_t)W ? slot - (uint32_t)W : slot;
                return make_int2(*global_ptr(xs + x), x >= unread ? *global_ptr(ring + slot) : 0);
            },
            [&](int32_t x, int2 v) {
                uint32_t slot = pos0 + (uint32_t)x;
                slot = slot >= (uint32_t)W ? slot - (uint32_t)W : slot;
                *global_ptr(ring + slot) = v.x;
                return (long long)v.x - (long long)v.y;
            });
        apply_emit(st, outs, g, f, f.sum0 + pre[0]);
        return;
    }
    // The old values [0, lold) and then the survivors [x_from, m) as one
    // sequence e: old value i sits in slot pos0 + i mod W (slots a window
    // that never filled has not reached hold 0 and are not read); survivors
    // at or past keep_from, the final window, go to the ring.  A round's
    // loads are all issued before any of its stores, and every old value
    // comes before every survivor, so no old value is read after its slot
    // was written.
    const int32_t keep_from = f.m - min(W, f.kg);
    const int32_t x_from = f.need_x ? 0 : keep_from;
    const int32_t lold = f.lold;
    const uint32_t slot0 =
        (uint32_t)(((int64_t)f.pos0 + f.kg - min(W, f.kg)) % (int64_t)W);  // of keep_from
    const bool sums = f.k > 0 && !f.whole;
    const int32_t q[3] = {sums ? lold + f.hi - x_from : 0, sums ? lold + f.lo - x_from : 0,
                          sums ? f.cb : 0};
    long long pre[3] = {0, 0, 0};
    apply_run<8>(
        0, lold + (f.m - x_from), q, pre,
        [&](int32_t e) {
            uint32_t slot = pos0 + (uint32_t)e;
            slot = slot >= (uint32_t)W ? slot - (uint32_t)W : slot;
            const int32_t *src = e < lold ? ring + slot : xs + (x_from + e - lold);
            return (e < lold && e < unread) ? 0 : *global_ptr(src);
        },
        [&](int32_t e, int32_t v) {
            const int32_t p = x_from + e - lold;
            if (e >= lold && p >= keep_from) {
                uint32_t slot = slot0 + (uint32_t)(p - keep_from);
                slot = slot >= (uint32_t)W ? slot - (uint32_t)W : slot;
                *global_ptr(ring + slot) = v;
            }
            return (long long)v;
        });
    const long long s = f.whole ? (long long)f.tb
                                : (f.c < W ? f.sum0 : 0LL) + pre[0] - pre[1] - pre[2];
    apply_emit(st, outs, g, f, s);
}

// LDS of a workgroup's big group: per batch its prefix sums at its points
// as the wave whose run holds the point found them (survivors to hi and to
// lo, old values to cb), and each wave's run sums (old values, survivors).
struct BigLds {
    long long pre[3][SB_K];
    long long tot[2][APPLY_THREADS / 64];
};

// Group g by a whole workgroup (its survivors plus old values read exceed
// APPLY_BUDGET): the window sums of apply_wave's general case, with the
// old values and then the survivors each cut into one run per wave; a
// point's prefix sum is its run's part plus the sums of the runs before.
__device__ void apply_big(const State &st, const SbBufs &sb, const SbBatches &in,
                          const Out *outs, uint32_t vmask, int g, BigLds &bl) {
    constexpr int NW = APPLY_THREADS / 64;
    const int lane = lane_id(), wid = (int)threadIdx.x >> 6;
    const int32_t W = st.W;
    int32_t A;
    int64_t B;
    apply_facts(st, sb, in.K, g, A, B);
    const ApplyFacts f = apply_unpack(A, B, vmask, W);
    if ((int)threadIdx.x < 3 * SB_K) (&bl.pre[0][0])[threadIdx.x] = 0;
    __syncthreads();
    int32_t *ring = st.ring + (int64_t)g * W;
    const int32_t *xs = sb.xs + f.gs;
    const int32_t unread = W - f.cnt0;
    const uint32_t pos0 = (uint32_t)f.pos0;
    const int32_t keep_from = f.m - min(W, f.kg);
    const int32_t x_from = f.need_x ? 0 : keep_from;
    const int32_t lold = f.lold;
    const bool sums = f.k > 0 && !f.whole;
    // runs of whole rounds: wave w takes [a + w * L, a + (w + 1) * L) of [a, z)
    auto run_of = [&](int32_t a, int32_t z, int w, int32_t &r0, int32_t &r1) {
        const int32_t L = (z - a + NW * 64 - 1) / (NW * 64) * 64;
        r0 = min(z, a + w * L);
        r1 = min(z, r0 + L);
    };
    int32_t r0, r1;
    run_of(0, lold, wid, r0, r1);
    {
        const int32_t q[1] = {sums ? f.cb : 0};
        long long pre[1] = {0};
        const long long t = apply_run<16>(
            r0, r1, q, pre,
            [&](int32_t i) {
                uint32_t slot = pos0 + (uint32_t)i;
                slot = slot >= (uint32_t)W ? slot - (uint32_t)W : slot;
                return i < unread ? 0 : *global_ptr(ring + slot);
            },
            [&](int32_t, int32_t v) { return (long long)v; });
        if (lane < SB_K && (uint32_t)(q[0] - 1 - r0) < (uint32_t)(r1 - r0)) bl.pre[2][lane] = pre[0];
        if (lane == 0) bl.tot[0][wid] = t;
    }
    __syncthreads();  // (every old value has been read: the ring may change now)
    run_of(x_from, f.m, wid, r0, r1);
    const uint32_t slot0 =
        (uint32_t)(((int64_t)f.pos0 + f.kg - min(W, f.kg)) % (int64_t)W);  // of keep_from
    {
        const int32_t q[2] = {sums ? f.hi : 0, sums ? f.lo : 0};
        long long pre[2] = {0, 0};
        const long long t = apply_run<16>(
            r0, r1, q, pre, [&](int32_t p) { return *global_ptr(xs + p); },
            [&](int32_t p, int32_t v) {
                if (p >= keep_from) {
                    uint32_t slot = slot0 + (uint32_t)(p - keep_from);
                    slot = slot >= (uint32_t)W ? slot - (uint32_t)W : slot;
                    *global_ptr(ring + slot) = v;
                }
                return (long long)v;
            });
#pragma unroll
        for (int j = 0; j < 2; ++j)
            if (lane < SB_K && (uint32_t)(q[j] - 1 - r0) < (uint32_t)(r1 - r0))
                bl.pre[j][lane] = pre[j];
        if (lane == 0) bl.tot[1][wid] = t;
    }
    __syncthreads();
    if (wid == 0) {
        // a point's prefix: its run's part plus the runs that end before it
        auto prefix = [&](int ph, int j, int32_t a, int32_t z, int32_t qp) {
            long long s = qp > a ? bl.pre[j][lane < SB_K ? lane : 0] : 0LL;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                int32_t w0, w1;
                run_of(a, z, w, w0, w1);
                s += w1 < qp ? bl.tot[ph][w] : 0LL;
            }
            return s;
        };
        const long long s =
            f.whole ? (long long)f.tb
                    : (f.c < W ? f.sum0 : 0LL) + prefix(1, 0, x_from, f.m, f.hi) -
                          prefix(1, 1, x_from, f.m, f.lo) - prefix(0, 2, 0, lold, f.cb);
        apply_emit(st, outs, g, f, s);
    }
    __syncthreads();
}

__global__ __launch_bounds__(APPLY_THREADS, 4) void k_sb_apply(State st, Scratch base, SbBufs sb,
                                                            SbBatches in, int32_t seq) {
    __shared__ BigLds bigl;
    __shared__ Out outs[SB_K];  // (indexed by lane: the argument's copy is per batch)
    const int K = in.K;
    const int G = (int)st.G;
    const int lane = lane_id();
#pragma unroll
    for (int b = 0; b < SB_K; ++b)
        if ((int)threadIdx.x == b) outs[b] = in.out[b];
    const uint32_t vmask = (uint32_t)ballot(lane < K && sb.sbad[lane < K ? lane : 0] != seq);
    __syncthreads();
    phase_mark(base, PHASE_SB_APPLY, 0);
    // The groups over APPLY_BUDGET by whole workgroups, the last min(nbig,
    // grid) ones; every other group by one wave of the workgroups before
    // those (of all of them when every workgroup has a big group), each wave
    // taking every NWV-th group, the next one's facts loaded while the
    // current one is worked on.
    const int nbig = sb.ntot[0];
    const int grid = (int)gridDim.x;
    const int nbw = min(nbig, grid);
    const int bw = grid - 1 - (int)blockIdx.x;  // this workgroup's place from the top
    for (int i = bw; i < nbig; i += grid) {
        apply_big(st, sb, in, outs, vmask, sb.big[i], bigl);
        if (i == bw) phase_mark(base, PHASE_SB_APPLY, 1);
    }
    phase_mark(base, PHASE_SB_APPLY, 2);
    const int wgs = nbw < grid ? grid - nbw : grid;  // workgroups that take wave groups
    if ((int)blockIdx.x >= wgs) {
        phase_mark(base, PHASE_SB_APPLY, 7);
        return;
    }
    const int NWV = wgs * (APPLY_THREADS / 64);
    int g = (int)blockIdx.x * (APPLY_THREADS / 64) + ((int)threadIdx.x >> 6);
    int32_t A0;
    int64_t B0;
    apply_facts(st, sb, K, g, A0, B0);
    for (; g < G; g += NWV) {
        int32_t A1;
        int64_t B1;
        apply_facts(st, sb, K, g + NWV, A1, B1);
        keep(A0);
        keep(B0);
        if (!__builtin_amdgcn_readlane(A0, AF_BIG))  // (else a workgroup's)
            apply_wave(st, sb, outs, vmask, g, A0, B0);
        A0 = A1;
        B0 = B1;
    }
    phase_mark(base, PHASE_SB_APPLY, 7);
}

// ------------------------------------------------------------ launchers --

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int64_t hist_blocks(int64_t n, int64_t G) {
    (void)G;
    return std::max<int64_t>(1, (n + HIST_TILE - 1) / HIST_TILE);
}

hipError_t launch_validate(const int32_t *keys, int64_t n, int64_t G, int32_t seq, Scratch sc,
                           hipStream_t s) {
    int64_t grid = (n + 4095) / 4096;
    grid = std::max<int64_t>(1, std::min<int64_t>(grid, 2048));
    hipLaunchKernelGGL(k_validate, dim3((unsigned)grid), dim3(256), 0, s, keys, n, G, seq, sc);
    return hipGetLastError();
}

hipError_t launch_hist(const int32_t *keys, int64_t n, int64_t G, Scratch sc, int32_t seq,
                       hipStream_t s) {
    if (G <= HIST_DIRECT_MAX_G) {
        const int64_t grid = hist_blocks(n, G);
        hipLaunchKernelGGL(k_hist_small, dim3((unsigned)grid), dim3(HIST_THREADS),
                           (size_t)G * 4, s, keys, n, aligned16(keys), (int32_t)G, sc, seq);
    } else {
        const int64_t tiles = std::max<int64_t>((n + HIST_HASH_TILE - 1) / HIST_HASH_TILE, 1);
        hipLaunchKernelGGL(k_hist_hash, dim3((unsigned)tiles), dim3(HIST_THREADS),
                           (size_t)2 * HIST_HASH_SLOTS * 4, s, keys, n, G, seq, sc);
    }
    return hipGetLastError();
}

hipError_t launch_plan(State st, Scratch sc, int32_t seq, int mode, int32_t workers,
                       hipStream_t s) {
    const int64_t G = st.G;
    if (plan_fused(G)) return hipSuccess;  // planned inside the pass
    if (G <= HIST_DIRECT_MAX_G) {
        hipLaunchKernelGGL(k_plan_small, dim3((unsigned)((G + PS_THREADS - 1) / PS_THREADS)),
                           dim3(PS_THREADS), 0, s, st, sc, seq, mode, workers);
        return hipGetLastError();
    }
    const int64_t nblk = (G + PLAN_CHUNK - 1) / PLAN_CHUNK;
    hipLaunchKernelGGL(k_plan_reduce, dim3((unsigned)nblk), dim3(PLAN_THREADS), 0, s, G, mode,
                       sc);
    if (nblk <= PLAN_SCAN_IN_BLOCK_MAX) {
        hipLaunchKernelGGL(k_plan_down<true>, dim3((unsigned)nblk), dim3(PLAN_THREADS), 0, s, st,
                           sc, seq, mode, workers, (int32_t)nblk);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(PLAN_THREADS), 0, s, (int32_t)nblk, st, sc, seq,
                       mode, workers);
    hipLaunchKernelGGL(k_plan_down<false>, dim3((unsigned)nblk), dim3(PLAN_THREADS), 0, s, st, sc,
                       seq, mode, workers, (int32_t)nblk);
    return hipGetLastError();
}

hipError_t launch_pass(const int32_t *keys, const int32_t *values, int64_t n, State st,
                       Scratch sc, int32_t seq, int mode, int32_t workers, hipStream_t s) {
    const int64_t tiles = (n + PASS_TILE - 1) / PASS_TILE;
    if (plan_fused(st.G))
        hipLaunchKernelGGL(k_pass<true>, dim3((unsigned)tiles), dim3(PASS_THREADS), 0, s, keys,
                           values, n, st, sc, seq, mode, workers);
    else
        hipLaunchKernelGGL(k_pass<false>, dim3((unsigned)tiles), dim3(PASS_THREADS), 0, s, keys,
                           values, n, st, sc, seq, mode, workers);
    return hipGetLastError();
}

int64_t update_grid(int64_t n, int mode, int32_t workers) {
    if (mode == MODE_STATIC) return (workers + STATIC_WORKERS_PER_WG - 1) / STATIC_WORKERS_PER_WG;
    const int64_t nb = (n + LIGHT_BUDGET - 1) / LIGHT_BUDGET + n / HEAVY_MIN + 1;
    // a whole number of workgroups per XCD
    return (std::max<int64_t>(1, std::min<int64_t>(nb, NB_MAX)) + XCDS - 1) / XCDS * XCDS;
}

bool can_fuse_hist(int64_t G, int mode) { return mode != MODE_STATIC && plan_fused(G); }

hipError_t launch_update(State st, Scratch sc, int64_t n, int mode, int32_t workers, Out out,
                         hipStream_t s, const int32_t *next_keys, int64_t next_n, Scratch next_sc,
                         int32_t next_seq) {
    const int tiles = (int)((n + PASS_TILE - 1) / PASS_TILE);
    const int64_t grid = update_grid(n, mode, workers);
    if (mode == MODE_STATIC) {
        hipLaunchKernelGGL(k_update_static, dim3((unsigned)grid), dim3(UPD_THREADS), 0, s, st, sc,
                           tiles, workers, out);
    } else {
        NextHist nh{};
        if (next_keys && next_n > 0 && can_fuse_hist(st.G, mode)) {
            nh.keys = next_keys;
            nh.n = next_n;
            nh.vec = aligned16(next_keys);
            // a whole number per XCD, so update workgroup u still runs on
            // XCD u mod 8 (tiles past the batch count nothing)
            nh.blocks = (int32_t)(((next_n + FH_TILE - 1) / FH_TILE + XCDS - 1) / XCDS * XCDS);
            nh.seq = next_seq;
            nh.sc = next_sc;
        }
        hipLaunchKernelGGL(k_update_balanced, dim3((unsigned)(grid + nh.blocks)),
                           dim3(UPD_THREADS), 0, s, st, sc, tiles, out, nh);
    }
    return hipGetLastError();
}

hipError_t launch_collect_touched(int64_t G, int32_t seq, Scratch sc, hipStream_t s) {
    const int64_t nblk = (G + PLAN_CHUNK - 1) / PLAN_CHUNK;
    hipLaunchKernelGGL(k_touch_reduce, dim3((unsigned)nblk), dim3(PLAN_THREADS), 0, s, G, seq,
                       sc);
    hipLaunchKernelGGL(k_touch_scan, dim3(1), dim3(PLAN_THREADS), 0, s, (int32_t)nblk, sc);
    hipLaunchKernelGGL(k_touch_write, dim3((unsigned)nblk), dim3(PLAN_THREADS), 0, s, G, seq, sc);
    return hipGetLastError();
}

hipError_t launch_emit(State st, Scratch sc, int64_t cap, Out out, hipStream_t s) {
    int64_t grid = (cap + EMIT_THREADS - 1) / EMIT_THREADS;
    grid = std::max<int64_t>(1, std::min<int64_t>(grid, 1024));
    hipLaunchKernelGGL(k_emit, dim3((unsigned)grid), dim3(EMIT_THREADS), 0, s, st, sc, out);
    return hipGetLastError();
}

__global__ void k_set_touched(int64_t *n_touched, int64_t v) { *n_touched = v; }

__global__ void k_bump_seq(int32_t *seqp) {
    if (threadIdx.x == 0) atomicAdd(seqp, 1);
}

__global__ void k_set_seq(int32_t *seqp, int32_t v) {
    if (threadIdx.x == 0) atomicExch(seqp, v);
}

hipError_t launch_set_touched(int64_t *n_touched, int64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_touched, dim3(1), dim3(1), 0, s, n_touched, v);
    return hipGetLastError();
}

hipError_t launch_bump_seq(Scratch sc, hipStream_t s) {
    hipLaunchKernelGGL(k_bump_seq, dim3(1), dim3(64), 0, s, sc.seqp);
    return hipGetLastError();
}

hipError_t launch_set_seq(Scratch sc, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_seq, dim3(1), dim3(64), 0, s, sc.seqp, v);
    return hipGetLastError();
}

hipError_t launch_reset_totals(Scratch sc, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_totals, dim3(1), dim3(1), 0, s, sc);
    return hipGetLastError();
}

// -------------------------------------------------- several batches --

hipError_t launch_sb_hist(State st, Scratch base, SbBufs sb, const SbBatches &in, int32_t seq,
                          hipStream_t s) {
    const int grid = in.htile0[in.K];
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sb_hist, dim3((unsigned)grid), dim3(SBH_THREADS),
                       (size_t)((st.G + 1) / 2) * 4, s, base, sb, in, (int32_t)st.G, seq);
    return hipGetLastError();
}

hipError_t launch_sb_plan(State st, Scratch base, SbBufs sb, const SbBatches &in, int32_t seq,
                          hipStream_t s) {
    const int64_t gs = (st.G + SBS_GROUPS - 1) / SBS_GROUPS;
    const int64_t gp = (st.G + SBP_THREADS - 1) / SBP_THREADS;
    hipLaunchKernelGGL(k_sb_sums, dim3((unsigned)gs), dim3(SBS_THREADS), 0, s, st, base, sb, in,
                       seq);
    hipLaunchKernelGGL(k_sb_plan, dim3((unsigned)gp, PLAN_SPLIT), dim3(SBP_THREADS), 0, s, st,
                       base, sb, in, seq);
    return hipGetLastError();
}

hipError_t launch_sb_pass(State st, Scratch base, SbBufs sb, const SbBatches &in, int32_t seq,
                          hipStream_t s) {
    const int tiles = in.ptile0[in.K];
    if (tiles <= 0) return hipSuccess;
    // one workgroup per CU (the reorder's LDS), each over a run of tiles
    const int grid = std::min(tiles, SB_PASS_GRID);
    hipLaunchKernelGGL(k_sb_pass, dim3((unsigned)grid), dim3(PASS_THREADS), 0, s, st, base, sb,
                       in, seq);
    return hipGetLastError();
}

hipError_t launch_sb_prep(State st, Scratch base, SbBufs sb, const SbBatches &in,
                          hipStream_t s) {
    // waves loop over the items (at most one per bucket of each batch, known
    // on the device only): a workgroup that finds none still costs its
    // dispatch, so the grid is what the device holds at once, not the bound
    int64_t items = 0;
    for (int b = 0; b < in.K; ++b)
        items += in.n[b] ? (in.n[b] + SB_LIGHT_BUDGET - 1) / SB_LIGHT_BUDGET + in.n[b] / SB_HEAVY_MIN + 1
                         : 0;
    const int64_t grid = std::max<int64_t>(
        1, std::min<int64_t>((items + UPD_THREADS / 64 - 1) / (UPD_THREADS / 64), SB_PREP_GRID));
    hipLaunchKernelGGL(k_sb_prep, dim3((unsigned)grid), dim3(UPD_THREADS), 0, s, st, base, sb,
                       in);
    return hipGetLastError();
}

hipError_t launch_sb_apply(State st, Scratch base, SbBufs sb, const SbBatches &in, int32_t seq,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_sb_apply, dim3(SB_APPLY_GRID), dim3(APPLY_THREADS), 0, s, st, base, sb,
                       in, seq);
    return hipGetLastError();
}

}  // namespace cq
