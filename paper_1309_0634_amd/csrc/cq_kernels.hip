// HIP kernels for gfx950 (CDNA4, wave64): one batch of the continuous
// sliding-window group-by aggregate.
//
// Per batch, in stream order:
//   k_hist     arrival tiles -> key histogram k[g]; flags keys outside
//              [0, G) (tuples are (id, attr), Section 3; a bad batch is
//              rejected whole);
//   k_plan_*   scans over the groups: light/heavy split, touched list,
//              light buckets packed by tuple count, heavy work items -- the
//              load balancer, decided from this batch's exact histogram
//              (the paper's coordinator moves groups between threads on the
//              CPU with a one-iteration delay, Section 3.1 and Section 4);
//   k_scatter  arrival tiles -> every tuple staged with its arrival index in
//              its group's segment (the paper's reordered data matrix,
//              Section 3.1, grouped by group instead of by thread); one
//              global reservation per (tile, group); heavy groups also get a
//              run descriptor per tile;
//   k_update_* the per-group phase: each group's surviving tuples (its last
//              W in arrival order) go to its ring slots; the evicted slot
//              values are subtracted and the new ones added (Section 3.2:
//              a full window discards its oldest value, nextPos moves on);
//   k_emit     (from cq_results) the touched groups' SUM, COUNT, AVG in
//              ascending id.
//
// The path is integer work bounded by memory traffic: no MFMA.
#include "cq_internal.h"
#include "cq.h"

namespace cq {

// ------------------------------------------------------------ utilities --

__device__ __forceinline__ int wave_incl_add(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_incl_max_u64(unsigned long long v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned long long t = __shfl_up(v, o, 64);
        if (lane >= o && t > v) v = t;
    }
    return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive block scan of F ints per thread; `lds` holds F * (waves) ints.
// Returns the block totals in `total`.  Contains barriers: call uniformly.
template <int F>
__device__ void block_excl_scan(int (&v)[F], int (&total)[F], int *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int incl[F];
#pragma unroll
    for (int f = 0; f < F; ++f) incl[f] = wave_incl_add(v[f]);
    if (lane == 63) {
#pragma unroll
        for (int f = 0; f < F; ++f) lds[wid * F + f] = incl[f];
    }
    __syncthreads();
    if (wid == 0) {
#pragma unroll
        for (int f = 0; f < F; ++f) {
            int x = lane < nw ? lds[lane * F + f] : 0;
            int s = wave_incl_add(x);
            if (lane < nw) lds[lane * F + f] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < F; ++f) {
        int before = wid > 0 ? lds[(wid - 1) * F + f] : 0;
        total[f] = lds[(nw - 1) * F + f];
        v[f] = before + incl[f] - v[f];
    }
    __syncthreads();
}

// Block sum of an int; `lds` holds >= waves ints.  Barriers inside.
__device__ int block_sum_int(int v, int *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    v = wave_sum_int(v);
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < nw; ++w) t += lds[w];
    __syncthreads();
    return t;
}

__device__ long long block_sum_ll(long long v, long long *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    v = wave_sum_ll(v);
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    long long t = 0;
    for (int w = 0; w < nw; ++w) t += lds[w];
    __syncthreads();
    return t;
}

// Inclusive max-scan of a[0, size) in LDS (unsigned 64-bit).  Each thread
// scans a contiguous piece, then pieces are combined across the block.
__device__ void block_incl_max_scan_u64(unsigned long long *a, int size,
                                        unsigned long long *lds_w) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nw = blockDim.x >> 6;
    const int per = (size + blockDim.x - 1) / blockDim.x;
    const int b0 = min(size, tid * per), b1 = min(size, b0 + per);
    unsigned long long m = 0;
    for (int i = b0; i < b1; ++i) {
        unsigned long long x = a[i];
        if (x > m) m = x;
        a[i] = m;
    }
    unsigned long long incl = wave_incl_max_u64(m);
    if (lane == 63) lds_w[wid] = incl;
    __syncthreads();
    unsigned long long before = 0;
    for (int w = 0; w < wid; ++w)
        if (lds_w[w] > before) before = lds_w[w];
    unsigned long long prev = __shfl_up(incl, 1, 64);
    if (lane > 0 && prev > before) before = prev;
    for (int i = b0; i < b1; ++i)
        if (a[i] < before) a[i] = before;
    __syncthreads();
    (void)nw;
}

// In-LDS bitonic sort, ascending, of key[0, P2) (P2 a power of two), with an
// optional int payload.  Barriers inside; P2 must be uniform.
template <bool PAYLOAD>
__device__ void bitonic_sort(unsigned long long *key, int32_t *val, int P2) {
    for (int k = 2; k <= P2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < (P2 >> 1); t += blockDim.x) {
                const int lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const int hi = lo + j;
                const bool asc = (lo & k) == 0;
                unsigned long long a = key[lo], b = key[hi];
                if ((a > b) == asc) {
                    key[lo] = b;
                    key[hi] = a;
                    if (PAYLOAD) {
                        int32_t x = val[lo];
                        val[lo] = val[hi];
                        val[hi] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Arrival-tile loader: item j of thread t is tuple base + 4*(j/4*256 + t) +
// j%4, so every wave reads 1 KiB contiguous per vector load.
__device__ __forceinline__ int64_t tile_index(int64_t base, int j) {
    return base + 4 * ((int64_t)(j >> 2) * TILE_THREADS + threadIdx.x) + (j & 3);
}

__device__ __forceinline__ void load_tile(const int32_t *__restrict__ p, int64_t base,
                                          int64_t n, bool vec, int32_t (&v)[ITEMS]) {
#pragma unroll
    for (int q = 0; q < ITEMS / 4; ++q) {
        const int64_t i0 = base + 4 * ((int64_t)q * TILE_THREADS + threadIdx.x);
        if (vec && i0 + 3 < n) {
            int4 x = *reinterpret_cast<const int4 *>(p + i0);
            v[4 * q + 0] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[4 * q + e] = (i0 + e < n) ? p[i0 + e] : 0;
        }
    }
}

// Open-addressing LDS hash: slot holding `key` (inserted if absent).  Keys
// are >= 0; empty slots hold -1.  At most TILE distinct keys per tile and
// HASH_SLOTS >= 2*TILE, so a free slot is always found.
__device__ __forceinline__ int hash_slot(int32_t *hk, int32_t key) {
    uint32_t h = ((uint32_t)key * 2654435761u) >> (32 - HASH_LOG);
    while (true) {
        int32_t prev = atomicCAS(&hk[h], -1, key);
        if (prev == -1 || prev == key) return (int)h;
        h = (h + 1) & (HASH_SLOTS - 1);
    }
}

// --------------------------------------------------------------- k_hist --
// One arrival tile per workgroup: count keys in LDS (indexed directly, or
// through the hash for large G), then one global atomic per distinct key.
template <bool DIRECT>
__global__ __launch_bounds__(TILE_THREADS) void k_hist(const int32_t *__restrict__ keys,
                                                       int64_t n, int64_t G, bool vec,
                                                       int32_t *__restrict__ k,
                                                       int32_t *__restrict__ flag) {
    extern __shared__ int32_t lds[];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    int32_t kv[ITEMS];
    load_tile(keys, base, n, vec, kv);
    int32_t *hk = lds, *hc = lds + HASH_SLOTS;
    if (DIRECT) {
        for (int g = tid; g < (int)G; g += TILE_THREADS) lds[g] = 0;
    } else {
        for (int s = tid; s < HASH_SLOTS; s += TILE_THREADS) {
            hk[s] = -1;
            hc[s] = 0;
        }
    }
    __syncthreads();
    int bad = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (tile_index(base, j) >= n) continue;
        const int32_t key = kv[j];
        if (key < 0 || (int64_t)key >= G) {
            bad = 1;
            continue;
        }
        if (DIRECT)
            atomicAdd(&lds[key], 1);
        else
            atomicAdd(&hc[hash_slot(hk, key)], 1);
    }
    if (__syncthreads_or(bad)) {
        if (tid == 0) atomicOr(flag, 1);
    }
    if (DIRECT) {
        for (int g = tid; g < (int)G; g += TILE_THREADS) {
            const int32_t c = lds[g];
            if (c) atomicAdd(&k[g], c);
        }
    } else {
        for (int s = tid; s < HASH_SLOTS; s += TILE_THREADS) {
            const int32_t key = hk[s];
            if (key >= 0) atomicAdd(&k[key], hc[s]);
        }
    }
}

// --------------------------------------------------------------- k_plan --
// Per group g with k_g tuples in this batch:
//   light (0 < k_g < HEAVY_MIN) -> field 0 (tuples), packed into buckets;
//   heavy (k_g >= HEAVY_MIN)    -> fields 1 (index), 2 (tuples), 4 (runs);
//   touched (k_g > 0)           -> field 3 (output position).
__device__ __forceinline__ void key_fields(int32_t kg, int32_t tiles, int (&f)[PLAN_FIELDS]) {
    const bool heavy = kg >= HEAVY_MIN;
    const bool light = kg > 0 && !heavy;
    f[0] = light ? kg : 0;
    f[1] = heavy ? 1 : 0;
    f[2] = heavy ? kg : 0;
    f[3] = kg > 0 ? 1 : 0;
    f[4] = heavy ? min(tiles, kg) : 0;
}

// Sums of the fields over this thread's PLAN_KPT consecutive groups.
__device__ void plan_thread_sums(const int32_t *__restrict__ k, int64_t g0, int64_t G,
                                 int32_t tiles, int (&f)[PLAN_FIELDS]) {
#pragma unroll
    for (int i = 0; i < PLAN_FIELDS; ++i) f[i] = 0;
    for (int i = 0; i < PLAN_KPT; ++i) {
        const int64_t g = g0 + i;
        if (g >= G) break;
        int x[PLAN_FIELDS];
        key_fields(k[g], tiles, x);
#pragma unroll
        for (int q = 0; q < PLAN_FIELDS; ++q) f[q] += x[q];
    }
}

// Write the per-group plan for this thread's groups, starting from the
// exclusive running values `run`; zero the histogram for the next batch.
__device__ void plan_thread_write(int32_t *__restrict__ k, int64_t g0, int64_t G,
                                  int32_t tiles, int (&run)[PLAN_FIELDS],
                                  int32_t light_total, const Scratch &sc) {
    for (int i = 0; i < PLAN_KPT; ++i) {
        const int64_t g = g0 + i;
        if (g >= G) break;
        const int32_t kg = k[g];
        k[g] = 0;
        int x[PLAN_FIELDS];
        key_fields(kg, tiles, x);
        sc.lpre[g] = run[0];
        sc.hcum[g] = run[1];
        if (kg > 0) sc.touched[run[3]] = (int32_t)g;
        if (x[0]) {
            sc.cursor[g] = run[0];
            // Light buckets: bucket m starts at the group whose staged range
            // [L, L + k_g) contains position m * LIGHT_BUDGET.
            const int32_t L = run[0];
            const int32_t m = (L + LIGHT_BUDGET - 1) / LIGHT_BUDGET;
            if ((int64_t)m * LIGHT_BUDGET <= (int64_t)L + kg - 1) sc.bkey[m] = (int32_t)g;
        } else if (x[1]) {
            const int32_t h = run[1];
            sc.hkey[h] = (int32_t)g;
            sc.hpre[h] = run[2];
            sc.hdb[h] = run[4];
            sc.hruns[h] = 0;
            sc.cursor[g] = light_total + run[2];
        }
#pragma unroll
        for (int q = 0; q < PLAN_FIELDS; ++q) run[q] += x[q];
    }
}

// Totals -> PlanTotals and sentinels; takes the bad-key flag of the batch.
__device__ void plan_publish(int (&tot)[PLAN_FIELDS], int64_t G, int32_t tiles,
                             const Scratch &sc) {
    const int32_t nl = (tot[0] + LIGHT_BUDGET - 1) / LIGHT_BUDGET;
    PlanTotals t;
    t.n_light_buckets = nl;
    t.n_heavy = tot[1];
    t.light_tuples = tot[0];
    t.heavy_tuples = tot[2];
    t.n_touched = tot[3];
    t.n_desc = tot[4];
    t.status = *sc.flag ? CQ_ERR_KEY_RANGE : 0;
    t.tiles = tiles;
    *sc.tot = t;
    *sc.flag = 0;
    sc.bkey[nl] = (int32_t)G;
    sc.lpre[G] = tot[0];
    sc.hcum[G] = tot[1];
    sc.hpre[tot[1]] = tot[2];
}

// Whole plan in one workgroup (G <= PLAN_CHUNK).
__global__ __launch_bounds__(PLAN_THREADS) void k_plan_single(int64_t G, int32_t tiles,
                                                              Scratch sc) {
    __shared__ int lds[PLAN_FIELDS * (PLAN_THREADS / 64)];
    const int64_t g0 = (int64_t)threadIdx.x * PLAN_KPT;
    int f[PLAN_FIELDS], tot[PLAN_FIELDS];
    plan_thread_sums(sc.k, g0, G, tiles, f);
    block_excl_scan<PLAN_FIELDS>(f, tot, lds);
    if (threadIdx.x == 0) plan_publish(tot, G, tiles, sc);
    plan_thread_write(sc.k, g0, G, tiles, f, tot[0], sc);
}

// Multi-block plan, phase 1: block sums.
__global__ __launch_bounds__(PLAN_THREADS) void k_plan_reduce(int64_t G, int32_t tiles,
                                                              Scratch sc) {
    __shared__ int lds[PLAN_FIELDS * (PLAN_THREADS / 64)];
    const int64_t g0 = (int64_t)blockIdx.x * PLAN_CHUNK + (int64_t)threadIdx.x * PLAN_KPT;
    int f[PLAN_FIELDS], tot[PLAN_FIELDS];
    plan_thread_sums(sc.k, g0, G, tiles, f);
    block_excl_scan<PLAN_FIELDS>(f, tot, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < PLAN_FIELDS; ++q) sc.partials[blockIdx.x * PLAN_FIELDS + q] = tot[q];
}

// Phase 2 (one workgroup): exclusive scan of the block sums, totals.
__global__ __launch_bounds__(PLAN_THREADS) void k_plan_scan(int32_t nblk, int64_t G,
                                                            int32_t tiles, Scratch sc) {
    __shared__ int lds[PLAN_FIELDS * (PLAN_THREADS / 64)];
    const int per = (nblk + PLAN_THREADS - 1) / PLAN_THREADS;
    const int b0 = min(nblk, (int)threadIdx.x * per), b1 = min(nblk, b0 + per);
    int f[PLAN_FIELDS] = {0, 0, 0, 0, 0}, tot[PLAN_FIELDS];
    for (int b = b0; b < b1; ++b)
        for (int q = 0; q < PLAN_FIELDS; ++q) f[q] += sc.partials[b * PLAN_FIELDS + q];
    block_excl_scan<PLAN_FIELDS>(f, tot, lds);
    for (int b = b0; b < b1; ++b)
        for (int q = 0; q < PLAN_FIELDS; ++q) {
            const int x = sc.partials[b * PLAN_FIELDS + q];
            sc.partials[b * PLAN_FIELDS + q] = f[q];
            f[q] += x;
        }
    if (threadIdx.x == 0) plan_publish(tot, G, tiles, sc);
}

// Phase 3: per-group outputs from the block offsets.
__global__ __launch_bounds__(PLAN_THREADS) void k_plan_down(int64_t G, int32_t tiles,
                                                            Scratch sc) {
    __shared__ int lds[PLAN_FIELDS * (PLAN_THREADS / 64)];
    const int64_t g0 = (int64_t)blockIdx.x * PLAN_CHUNK + (int64_t)threadIdx.x * PLAN_KPT;
    int f[PLAN_FIELDS], tot[PLAN_FIELDS];
    plan_thread_sums(sc.k, g0, G, tiles, f);
    block_excl_scan<PLAN_FIELDS>(f, tot, lds);
#pragma unroll
    for (int q = 0; q < PLAN_FIELDS; ++q) f[q] += sc.partials[blockIdx.x * PLAN_FIELDS + q];
    plan_thread_write(sc.k, g0, G, tiles, f, sc.tot->light_tuples, sc);
}

// ------------------------------------------------------------ k_scatter --
// One arrival tile per workgroup.  Count the tile's tuples per group in LDS
// (the returned old count is the tuple's place inside the tile's run), then
// reserve each group's run with one global atomic on its cursor, and stage
// (arrival index, value) pairs there.  Runs of heavy groups are recorded as
// descriptors so the per-group phase can find the group's last tuples.
template <bool DIRECT>
__global__ __launch_bounds__(TILE_THREADS) void k_scatter(const int32_t *__restrict__ keys,
                                                          const int32_t *__restrict__ values,
                                                          int64_t n, int64_t G, bool vec,
                                                          Scratch sc) {
    if (sc.tot->status) return;
    extern __shared__ int32_t lds[];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    int32_t kv[ITEMS], vv[ITEMS], loc[ITEMS], slot[ITEMS];
    load_tile(keys, base, n, vec, kv);
    load_tile(values, base, n, vec, vv);
    int32_t *hk = lds, *hc = lds + HASH_SLOTS;
    if (DIRECT) {
        for (int g = tid; g < (int)G; g += TILE_THREADS) lds[g] = 0;
    } else {
        for (int s = tid; s < HASH_SLOTS; s += TILE_THREADS) {
            hk[s] = -1;
            hc[s] = 0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (tile_index(base, j) >= n) continue;
        if (DIRECT) {
            slot[j] = kv[j];
            loc[j] = atomicAdd(&lds[kv[j]], 1);
        } else {
            slot[j] = hash_slot(hk, kv[j]);
            loc[j] = atomicAdd(&hc[slot[j]], 1);
        }
    }
    __syncthreads();
    const int nslots = DIRECT ? (int)G : HASH_SLOTS;
    int32_t *cnt = DIRECT ? lds : hc;
    for (int s = tid; s < nslots; s += TILE_THREADS) {
        const int32_t c = cnt[s];
        if (!c) continue;
        const int32_t g = DIRECT ? s : hk[s];
        const int32_t start = atomicAdd(&sc.cursor[g], c);
        if (sc.lpre[g + 1] == sc.lpre[g]) {  // not light: heavy
            const int32_t h = sc.hcum[g];
            const int32_t d = atomicAdd(&sc.hruns[h], 1);
            sc.desc[sc.hdb[h] + d] =
                make_int2(start, (int32_t)(blockIdx.x << RUN_COUNT_BITS) | (c - 1));
        }
        cnt[s] = start;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = tile_index(base, j);
        if (i >= n) continue;
        sc.sdat[cnt[slot[j]] + loc[j]] = make_int2((int32_t)i, vv[j]);
    }
}

// ------------------------------------------------------------- k_update --
// Shared memory carved per path (bytes).
constexpr int SMEM_BYTES = 57408;
// light path
constexpr int L_SK = 0;                       // u64[LCAP] (group << 32 | arrival)
constexpr int L_SV = L_SK + 8 * LCAP;         // i32[LCAP] values
constexpr int L_SEG = L_SV + 4 * LCAP;        // u64[LCAP] (group+1 << 32 | first pos)
constexpr int L_ACC = L_SEG + 8 * LCAP;       // i64[LCAP] per-group sum deltas
static_assert(L_ACC + 8 * LCAP <= SMEM_BYTES, "light LDS");
// heavy path
constexpr int HCH = TILE;                      // elements staged per chunk
constexpr int H_BUF = 0;                       // u64[HCH] (arrival << 32 | value)
constexpr int H_DC = H_BUF + 8 * HCH;          // int2[DESC_CACHE]
constexpr int H_LIST = H_DC + 8 * DESC_CACHE;  // int2[HCH] runs of the chunk
constexpr int H_LOFF = H_LIST + 8 * HCH;       // i32[HCH + 1] run offsets
static_assert(H_LOFF + 4 * (HCH + 1) + 16 <= SMEM_BYTES, "heavy LDS");

__device__ __forceinline__ void finalize_group(const State &st, int32_t g, int64_t kg,
                                               long long delta) {
    const int64_t c = (int64_t)st.cnt[g] + kg;
    st.cnt[g] = (int32_t)(c < st.W ? c : st.W);
    st.pos[g] = (int32_t)(((uint32_t)st.pos[g] + (uint32_t)kg) % (uint32_t)st.W);
    st.sum[g] += delta;
}

// Light groups [a, b): their staged tuples are contiguous, [lpre[a],
// lpre[b]), fewer than LCAP.  Sort each group's tuples by arrival index in
// LDS, then every tuple among the group's last W goes to ring slot
// (pos + rank) mod W, adding (new - old slot value) to the group's sum.
__device__ int light_chunk(int32_t a, int32_t b, const State &st, const Scratch &sc,
                           char *smem, unsigned long long *lds_w) {
    const int tid = threadIdx.x;
    const int32_t s0 = sc.lpre[a];
    const int size = sc.lpre[b] - s0;
    if (size <= 0) return 0;
    if (size > LCAP) {  // impossible for a well-formed plan
        if (threadIdx.x == 0) atomicOr(sc.fault, FAULT_LIGHT_SIZE);
        return 0;
    }
    unsigned long long *sk = reinterpret_cast<unsigned long long *>(smem + L_SK);
    int32_t *sv = reinterpret_cast<int32_t *>(smem + L_SV);
    unsigned long long *seg = reinterpret_cast<unsigned long long *>(smem + L_SEG);
    long long *acc = reinterpret_cast<long long *>(smem + L_ACC);
    const int P2 = next_pow2(size);
    for (int p = tid; p < size; p += blockDim.x) {
        seg[p] = 0;
        acc[p] = 0;
    }
    __syncthreads();
    // mark where each light group's staged range starts ...
    for (int32_t g = a + tid; g < b; g += blockDim.x) {
        const int32_t l0 = sc.lpre[g], l1 = sc.lpre[g + 1];
        if (l1 > l0)
            seg[l0 - s0] = ((unsigned long long)(uint32_t)(g - a + 1) << 32) | (uint32_t)(l0 - s0);
    }
    __syncthreads();
    // ... and spread the mark over the range
    block_incl_max_scan_u64(seg, size, lds_w);
    for (int p = tid; p < P2; p += blockDim.x) {
        if (p < size) {
            const int2 e = sc.sdat[s0 + p];
            const uint32_t gl = (uint32_t)(seg[p] >> 32) - 1;
            sk[p] = ((unsigned long long)gl << 32) | (uint32_t)e.x;
            sv[p] = e.y;
        } else {
            sk[p] = ~0ull;
        }
    }
    __syncthreads();
    bitonic_sort<true>(sk, sv, P2);
    const int32_t W = st.W;
    for (int p = tid; p < size; p += blockDim.x) {
        const int32_t g = a + (int32_t)(sk[p] >> 32);
        const int p0 = (int)(uint32_t)seg[p];
        const int32_t kg = sc.lpre[g + 1] - sc.lpre[g];
        const int32_t r = p - p0;
        const int32_t need = kg < W ? kg : W;
        if (r >= kg - need) {
            const uint32_t slot = ((uint32_t)st.pos[g] + (uint32_t)r) % (uint32_t)W;
            int32_t *cell = st.ring + (int64_t)g * W + slot;
            const int32_t old = *cell;
            const int32_t v = sv[p];
            *cell = v;
            atomicAdd(reinterpret_cast<unsigned long long *>(&acc[p0]),
                      (unsigned long long)((long long)v - (long long)old));
        }
    }
    __syncthreads();
    for (int p = tid; p < size; p += blockDim.x) {
        const unsigned long long s = seg[p];
        const int p0 = (int)(uint32_t)s;
        if (p == p0) {
            const int32_t g = a + (int32_t)(s >> 32) - 1;
            finalize_group(st, g, sc.lpre[g + 1] - sc.lpre[g], acc[p]);
        }
    }
    __syncthreads();
    return size;
}

// Tuples of heavy item i staged in tiles >= tau.
__device__ int heavy_tail_count(int32_t tau, int nd, bool cached, const int2 *dc,
                                const int2 *D, int *lds_i) {
    int s = 0;
    for (int d = threadIdx.x; d < nd; d += blockDim.x) {
        const int2 x = cached ? dc[d] : D[d];
        if ((x.y >> RUN_COUNT_BITS) >= tau) s += (x.y & ((1 << RUN_COUNT_BITS) - 1)) + 1;
    }
    return block_sum_int(s, lds_i);
}

// Heavy group (k_g >= HEAVY_MIN): only its last min(k_g, W) tuples matter.
// Walk its runs from the last arrival tile backwards in chunks of at most
// one tile's worth of tuples, sort each chunk by arrival index, and write
// the survivors.  Cost is bounded by the window plus one tile, whatever k_g.
__device__ int heavy_item(int32_t i, const State &st, const Scratch &sc, int32_t tiles,
                          char *smem, int *lds_i, long long *lds_ll) {
    const int tid = threadIdx.x;
    const int32_t h = sc.hkey[i];
    const int32_t kh = sc.hpre[i + 1] - sc.hpre[i];
    const int32_t W = st.W;
    const int32_t need = kh < W ? kh : W;
    const int nd = sc.hruns[i];
    const int2 *D = sc.desc + sc.hdb[i];
    unsigned long long *buf = reinterpret_cast<unsigned long long *>(smem + H_BUF);
    int2 *dc = reinterpret_cast<int2 *>(smem + H_DC);
    int2 *list = reinterpret_cast<int2 *>(smem + H_LIST);
    int32_t *loff = reinterpret_cast<int32_t *>(smem + H_LOFF);
    int32_t *nlist = loff + HCH + 1;
    const bool cached = nd <= DESC_CACHE;
    if (cached)
        for (int d = tid; d < nd; d += blockDim.x) dc[d] = D[d];
    __syncthreads();
    const int32_t pos_h = st.pos[h];
    long long acc = 0;
    int done = 0;
    int32_t hi = tiles, s_hi = 0;
    for (int guard = 0; s_hi < need && hi > 0 && guard <= tiles; ++guard) {
        // smallest tau with (tuples in tiles [tau, hi)) <= HCH
        int32_t lo_t = 0, hi_t = hi - 1;
        while (lo_t < hi_t) {
            const int32_t mid = (lo_t + hi_t) >> 1;
            if (heavy_tail_count(mid, nd, cached, dc, D, lds_i) - s_hi <= HCH)
                hi_t = mid;
            else
                lo_t = mid + 1;
        }
        const int32_t tau = lo_t;
        const int32_t s_tau = heavy_tail_count(tau, nd, cached, dc, D, lds_i);
        const int C = s_tau - s_hi;
        if (C <= 0 || C > HCH) {  // impossible for a well-formed plan
            if (tid == 0) atomicOr(sc.fault, FAULT_HEAVY_CHUNK);
            break;
        }
        // runs of the chunk
        if (tid == 0) *nlist = 0;
        __syncthreads();
        for (int d = tid; d < nd; d += blockDim.x) {
            const int2 x = cached ? dc[d] : D[d];
            const int32_t t = x.y >> RUN_COUNT_BITS;
            if (t >= tau && t < hi)
                list[atomicAdd(nlist, 1)] = make_int2(x.x, (x.y & ((1 << RUN_COUNT_BITS) - 1)) + 1);
        }
        __syncthreads();
        const int nl = *nlist;
        {   // offsets of the runs inside the chunk
            const int per = (nl + blockDim.x - 1) / blockDim.x;
            const int b0 = min(nl, tid * per), b1 = min(nl, b0 + per);
            int f[1] = {0}, t[1];
            for (int r = b0; r < b1; ++r) f[0] += list[r].y;
            block_excl_scan<1>(f, t, lds_i);
            for (int r = b0; r < b1; ++r) {
                loff[r] = f[0];
                f[0] += list[r].y;
            }
            if (tid == 0) loff[nl] = t[0];
        }
        __syncthreads();
        const int P2 = next_pow2(C);
        for (int e = tid; e < P2; e += blockDim.x) {
            if (e < C) {
                int lo = 0, up = nl - 1;  // run r with loff[r] <= e < loff[r+1]
                while (lo < up) {
                    const int mid = (lo + up + 1) >> 1;
                    if (loff[mid] <= e) lo = mid; else up = mid - 1;
                }
                const int2 x = sc.sdat[list[lo].x + (e - loff[lo])];
                buf[e] = ((unsigned long long)(uint32_t)x.x << 32) | (uint32_t)x.y;
            } else {
                buf[e] = ~0ull;
            }
        }
        __syncthreads();
        bitonic_sort<false>(buf, nullptr, P2);
        const int32_t rank0 = kh - s_tau;
        for (int p = tid; p < C; p += blockDim.x) {
            const int32_t rank = rank0 + p;
            if (rank >= kh - need) {
                const int32_t v = (int32_t)(uint32_t)buf[p];
                const uint32_t slot = ((uint32_t)pos_h + (uint32_t)rank) % (uint32_t)W;
                int32_t *cell = st.ring + (int64_t)h * W + slot;
                const int32_t old = *cell;
                *cell = v;
                acc += (long long)v - (long long)old;
            }
        }
        __syncthreads();
        done += C;
        s_hi = s_tau;
        hi = tau;
    }
    const long long delta = block_sum_ll(acc, lds_ll);
    if (tid == 0) finalize_group(st, h, kh, delta);
    __syncthreads();
    return done;
}

__device__ __forceinline__ void trace_begin(unsigned long long &t0) { t0 = wall_clock64(); }

__device__ __forceinline__ void trace_end(int64_t *trace, unsigned long long t0,
                                          int64_t tuples, int64_t items) {
    if (!trace || threadIdx.x != 0) return;
    const unsigned long long t1 = wall_clock64();
    const uint32_t hwid = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4);
    const uint32_t xcc = __builtin_amdgcn_s_getreg((15 << 11) | (0 << 6) | 20);
    int64_t *r = trace + 6 * (int64_t)blockIdx.x;
    r[0] = hwid;
    r[1] = xcc;
    r[2] = (int64_t)t0;
    r[3] = (int64_t)t1;
    r[4] = tuples;
    r[5] = items;
}

// Balanced assignment: work items are the plan's light buckets followed by
// the heavy groups; workgroups stride over them.
__global__ __launch_bounds__(UPD_THREADS) void k_update_balanced(State st, Scratch sc,
                                                                 int32_t tiles) {
    __shared__ __align__(16) char smem[SMEM_BYTES];
    __shared__ int lds_i[64];
    __shared__ long long lds_ll[16];
    __shared__ unsigned long long lds_w[16];
    unsigned long long t0;
    trace_begin(t0);
    int64_t tuples = 0, items = 0;
    if (!sc.tot->status) {
        const int32_t nl = sc.tot->n_light_buckets;
        const int32_t total = nl + sc.tot->n_heavy;
        for (int32_t it = blockIdx.x; it < total; it += gridDim.x) {
            if (it < nl)
                tuples += light_chunk(sc.bkey[it], sc.bkey[it + 1], st, sc, smem, lds_w);
            else
                tuples += heavy_item(it - nl, st, sc, tiles, smem, lds_i, lds_ll);
            ++items;
        }
    }
    trace_end(sc.trace, t0, tuples, items);
}

// Static assignment: worker w owns groups [w*G/P, (w+1)*G/P) and handles all
// of them itself -- light groups in LDS-sized pieces, then its heavy groups.
__global__ __launch_bounds__(UPD_THREADS) void k_update_static(State st, Scratch sc,
                                                               int32_t tiles, int32_t workers) {
    __shared__ __align__(16) char smem[SMEM_BYTES];
    __shared__ int lds_i[64];
    __shared__ long long lds_ll[16];
    __shared__ unsigned long long lds_w[16];
    unsigned long long t0;
    trace_begin(t0);
    int64_t tuples = 0, items = 0;
    if (!sc.tot->status) {
        const int64_t G = st.G;
        const int32_t g0 = (int32_t)(G * blockIdx.x / workers);
        const int32_t g1 = (int32_t)(G * (blockIdx.x + 1) / workers);
        int32_t a = g0;
        while (a < g1) {
            // largest b in (a, g1] whose light tuples [lpre[a], lpre[b]) fit
            int32_t lo = a + 1, hi = g1;
            const int32_t la = sc.lpre[a];
            while (lo < hi) {
                const int32_t mid = lo + (hi - lo + 1) / 2;
                if (sc.lpre[mid] - la <= LCAP) lo = mid; else hi = mid - 1;
            }
            tuples += light_chunk(a, lo, st, sc, smem, lds_w);
            ++items;
            a = lo;
        }
        for (int32_t i = sc.hcum[g0]; i < sc.hcum[g1]; ++i) {
            tuples += heavy_item(i, st, sc, tiles, smem, lds_i, lds_ll);
            ++items;
        }
    }
    trace_end(sc.trace, t0, tuples, items);
}

// --------------------------------------------------------------- k_emit --
__global__ __launch_bounds__(EMIT_THREADS) void k_emit(State st, Scratch sc, int32_t *ids,
                                                       int64_t *sums, int32_t *counts,
                                                       double *avgs, int64_t *n_touched) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t status = sc.tot->status;
    if (status) {
        if (gid == 0) *n_touched = status;
        return;
    }
    const int32_t nt = sc.tot->n_touched;
    if (gid == 0) *n_touched = nt;
    for (int64_t j = gid; j < nt; j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = sc.touched[j];
        const int64_t s = st.sum[g];
        const int32_t c = st.cnt[g];
        if (ids) ids[j] = g;
        if (sums) sums[j] = s;
        if (counts) counts[j] = c;
        if (avgs) avgs[j] = (double)s / (double)c;
    }
}

__global__ void k_reset_totals(Scratch sc) {
    PlanTotals t = {0, 0, 0, 0, 0, 0, 0, 0};
    *sc.tot = t;
}

// ------------------------------------------------------------ launchers --

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

hipError_t launch_hist(const int32_t *keys, int64_t n, int64_t G, Scratch sc, hipStream_t s) {
    const int64_t tiles = (n + TILE - 1) / TILE;
    const bool direct = G <= DIRECT_MAX_G;
    const size_t lds = direct ? (size_t)G * 4 : (size_t)2 * HASH_SLOTS * 4;
    if (direct)
        hipLaunchKernelGGL(k_hist<true>, dim3((unsigned)tiles), dim3(TILE_THREADS), lds, s, keys,
                           n, G, aligned16(keys), sc.k, sc.flag);
    else
        hipLaunchKernelGGL(k_hist<false>, dim3((unsigned)tiles), dim3(TILE_THREADS), lds, s, keys,
                           n, G, aligned16(keys), sc.k, sc.flag);
    return hipGetLastError();
}

hipError_t launch_plan(int64_t G, int32_t tiles, Scratch sc, hipStream_t s) {
    const int64_t nblk = (G + PLAN_CHUNK - 1) / PLAN_CHUNK;
    if (nblk == 1) {
        hipLaunchKernelGGL(k_plan_single, dim3(1), dim3(PLAN_THREADS), 0, s, G, tiles, sc);
    } else {
        hipLaunchKernelGGL(k_plan_reduce, dim3((unsigned)nblk), dim3(PLAN_THREADS), 0, s, G,
                           tiles, sc);
        hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(PLAN_THREADS), 0, s, (int32_t)nblk, G,
                           tiles, sc);
        hipLaunchKernelGGL(k_plan_down, dim3((unsigned)nblk), dim3(PLAN_THREADS), 0, s, G,
                           tiles, sc);
    }
    return hipGetLastError();
}

hipError_t launch_scatter(const int32_t *keys, const int32_t *values, int64_t n, int64_t G,
                          Scratch sc, hipStream_t s) {
    const int64_t tiles = (n + TILE - 1) / TILE;
    const bool direct = G <= DIRECT_MAX_G;
    const bool vec = aligned16(keys) && aligned16(values);
    const size_t lds = direct ? (size_t)G * 4 : (size_t)2 * HASH_SLOTS * 4;
    if (direct)
        hipLaunchKernelGGL(k_scatter<true>, dim3((unsigned)tiles), dim3(TILE_THREADS), lds, s,
                           keys, values, n, G, vec, sc);
    else
        hipLaunchKernelGGL(k_scatter<false>, dim3((unsigned)tiles), dim3(TILE_THREADS), lds, s,
                           keys, values, n, G, vec, sc);
    return hipGetLastError();
}

int64_t update_grid(int64_t n, int mode, int32_t workers) {
    if (mode == CQ_PARTITION_STATIC) return workers;
    const int64_t items = (n + LIGHT_BUDGET - 1) / LIGHT_BUDGET + n / HEAVY_MIN + 1;
    return items < UPD_MAX_GRID ? items : UPD_MAX_GRID;
}

hipError_t launch_update(State st, Scratch sc, int64_t n, int32_t tiles, int mode,
                         int32_t workers, hipStream_t s) {
    const int64_t grid = update_grid(n, mode, workers);
    if (mode == CQ_PARTITION_STATIC)
        hipLaunchKernelGGL(k_update_static, dim3((unsigned)grid), dim3(UPD_THREADS), 0, s, st, sc,
                           tiles, workers);
    else
        hipLaunchKernelGGL(k_update_balanced, dim3((unsigned)grid), dim3(UPD_THREADS), 0, s, st,
                           sc, tiles);
    return hipGetLastError();
}

hipError_t launch_emit(State st, Scratch sc, int64_t cap, int32_t *ids, int64_t *sums,
                       int32_t *counts, double *avgs, int64_t *n_touched, hipStream_t s) {
    int64_t grid = (cap + EMIT_THREADS - 1) / EMIT_THREADS;
    if (grid < 1) grid = 1;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)grid), dim3(EMIT_THREADS), 0, s, st, sc, ids, sums,
                       counts, avgs, n_touched);
    return hipGetLastError();
}

hipError_t launch_reset_totals(Scratch sc, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_totals, dim3(1), dim3(1), 0, s, sc);
    return hipGetLastError();
}

}  // namespace cq
