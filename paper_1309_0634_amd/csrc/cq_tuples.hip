// HIP kernel for gfx950: per-tuple results of one planned and reordered
// sub-batch -- the aggregate the paper recomputes after every insertion
// (Section 5.1: the whole window is scanned after each new tuple; the last
// experiment of Section 5.2 scans it ten times).
//
// The launch sits between the reorder pass and the update, so the window
// store still holds the state from before the sub-batch.  For a group g
// with ring pointer p (the slot of its next write) and its tuples of this
// sub-batch v_0 .. v_{k-1} in arrival order, let
//   seq[x]     = ring[g][(p + x) mod W] for 0 <= x < W: the slot that
//                insertion x overwrites (slots never written hold 0), and
//   seq[W + j] = v_j.
// The window right after v_r entered is seq[r+1 .. W+r]: W entries, zeros
// standing for values never written.  Its SUM is the sum of that range and
// its COUNT min(W, count before the sub-batch + r + 1).
//   passes = 0 : SUM = (sum before) + sum over j <= r of (v_j - seq[j]),
//                the incremental form, exact in integers;
//   passes >= 1: the range is summed from scratch, `passes` times, each
//                pass reading the window again.
// Either way the results are identical integers.
//
// Work items: every light bucket of the plan (consecutive groups, at most
// LIGHT_CAP tuples) and every PT_CH ranks of every heavy group, so a hot
// group is spread over many workgroups.  A light bucket's tuples arrive
// bucket-sorted per tile; an LDS sort on (group, arrival position) puts
// every group's tuples together in rank order.  A heavy group's tuples are
// its runs in tile order, already in rank order.
#include <climits>

#include "cq.h"
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

namespace {

constexpr int PT_THREADS = 256;
constexpr int PT_GRID_MAX = 2048;

// LDS layout (bytes)
constexpr int T_RS = 0;                                  // i32[PASS_TILES_MAX]
constexpr int T_RP = T_RS + 4 * PASS_TILES_MAX;          // i32[PASS_TILES_MAX + 4]
constexpr int T_HC = T_RP + 4 * (PASS_TILES_MAX + 4);    // i32[NB_MAX + 4] heavy item prefix
constexpr int T_RED = T_HC + 4 * (NB_MAX + 4);           // scan scratch
constexpr int T_W = T_RED + 8 * 64;                      // work area
// light bucket: sort keys, values, arrival indices (i32[LIGHT_CAP] each),
// prefix sums (i64[LIGHT_CAP])
constexpr int L_CK = T_W;
constexpr int L_V = L_CK + 4 * LIGHT_CAP;
constexpr int L_I = L_V + 4 * LIGHT_CAP;
constexpr int L_PS = L_I + 4 * LIGHT_CAP;
constexpr int L_END = L_PS + 8 * LIGHT_CAP;
// heavy item: a piece of seq (i32), arrival indices of ranks [r0, r1)
// (i32), prefix sums (i64)
constexpr int H_SPAN = PT_CH + PT_WMAX;
constexpr int H_V = T_W;
constexpr int H_I = H_V + 4 * H_SPAN;
constexpr int H_PS = H_I + 4 * PT_CH;
constexpr int H_END = H_PS + 8 * H_SPAN;
constexpr int T_BYTES = L_END > H_END ? L_END : H_END;
static_assert(LIGHT_CAP <= 1024, "10-bit arrival positions in the light sort key");
static_assert(LIGHT_CAP % PT_THREADS == 0, "whole positions per thread");
static_assert(CQ_TUPLE_MAX_GROUPS <= (1 << 21), "group offsets fit the light sort key");

// Inclusive scan of a[0, m) (int64, in LDS, in place); each thread scans a
// contiguous piece.  `red` holds one int64 per wave.  Barriers inside.
__device__ void block_incl_scan_ll(long long *a, int m, long long *red) {
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int per = (m + (int)blockDim.x - 1) / (int)blockDim.x;
    const int b0 = min(m, tid * per), b1 = min(m, b0 + per);
    long long s = 0;
    for (int i = b0; i < b1; ++i) {
        s += a[i];
        a[i] = s;
    }
    long long x = s;  // inclusive over the wave's threads
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const long long y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) red[wv] = x;
    __syncthreads();
    long long off = x - s;
    for (int w = 0; w < wv; ++w) off += red[w];
    for (int i = b0; i < b1; ++i) a[i] += off;
    __syncthreads();
}

// Ascending bitonic sort of a[0, m) in LDS, m a power of two.  Barriers
// inside.
__device__ void bitonic_sort(int32_t *a, int m) {
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < m; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t x = a[i], y = a[l];
                    if ((x > y) == ((i & k) == 0)) {
                        a[i] = y;
                        a[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Slot x of group g's eviction order (the slot insertion x overwrites).
__device__ __forceinline__ int32_t old_slot(const int32_t *row, int32_t po, int x, int32_t W) {
    return row[((uint32_t)po + (uint32_t)x) % (uint32_t)W];
}

// Sum of n int32 values at p, in four independent fp64 accumulators.
// Every partial sum is an integer of magnitude below W * 2^31 <= 2^41, so
// each addition is exact in binary64 whatever the order: the total is the
// exact integer.  (The int64 form needs three dependent integer operations
// per value; this needs a conversion and an add, in four chains.)
__device__ __forceinline__ void sum_run(const int32_t *p, int n, double (&acc)[4]) {
    int i = 0;
    for (; i + 32 <= n; i += 32) {  // 32 loads in flight before the adds
        int32_t t[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) t[u] = p[i + u];
#pragma unroll
        for (int u = 0; u < 32; ++u) acc[u & 3] += (double)t[u];
    }
    for (; i < n; ++i) acc[i & 3] += (double)p[i];
}

__device__ __forceinline__ void put(const PtOut &out, int32_t i, long long s, int32_t c) {
    if (out.sums) out.sums[i] = s;
    if (out.counts) out.counts[i] = c;
    if (out.avgs) out.avgs[i] = (double)s / (double)c;
}

// Light bucket b: groups [bstart[b], bstart[b+1]), tuples in light-prefix
// space [lpre[a], lpre[z]).
__device__ void light_item(int b, int NB, int tiles, const State &st, const Scratch &sc,
                           const PtOut &out, char *smem) {
    const int tid = threadIdx.x;
    int32_t *rs = reinterpret_cast<int32_t *>(smem + T_RS);
    int32_t *rp = reinterpret_cast<int32_t *>(smem + T_RP);
    int *red = reinterpret_cast<int *>(smem + T_RED);
    int32_t *ck = reinterpret_cast<int32_t *>(smem + L_CK);
    int32_t *lv = reinterpret_cast<int32_t *>(smem + L_V);
    int32_t *li = reinterpret_cast<int32_t *>(smem + L_I);
    long long *ps = reinterpret_cast<long long *>(smem + L_PS);
    const int32_t W = st.W;
    // the run rows depend on b alone: they are in flight while the bucket's
    // light prefix is read (the bounds are issued first: loads complete in
    // order, so waiting on them does not wait on the rows)
    const int32_t a = sc.bstart[b], z = sc.bstart[b + 1];
    RunRows<PT_THREADS> rr;
    runs_load<PT_THREADS>(sc, b, NB, tiles, rr);
    const int32_t s0 = sc.lpre[a];
    const int size = sc.lpre[z] - s0;
    const int total = runs_store<PT_THREADS>(tiles, rr, rs, rp, red);
    if (size <= 0) return;
    if (size > LIGHT_CAP || total != size) {
        if (tid == 0) atomicOr(sc.fault, FAULT_TUPLE_RUNS);
        return;
    }
    int m = 1;
    while (m < size) m <<= 1;
    constexpr int PPT = LIGHT_CAP / PT_THREADS;
    {
        // all of a thread's gathers are issued before any is used
        // (positions past the bucket are clamped onto its last one)
        // (the run searches first: a search is a loop, and loads issued
        // before one would be waited on where it starts)
        int2 ge[PPT];
        int32_t gi[PPT], gp[PPT];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int pc = min(tid + u * PT_THREADS, size - 1);
            const int r = upper_run(rp, tiles, pc);
            gp[u] = rs[r] + (pc - rp[r]);
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            ge[u] = sc.sdat[gp[u]];
            gi[u] = sc.sidx[gp[u]];
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            keep(ge[u].x);
            keep(ge[u].y);
            keep(gi[u]);
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int p = tid + u * PT_THREADS;
            if (p < size) {
                lv[p] = ge[u].y;
                li[p] = gi[u];
                ck[p] = ((ge[u].x - a) << 10) | p;
            } else if (p < m) {
                ck[p] = INT_MAX;
            }
        }
    }
    __syncthreads();
    bitonic_sort(ck, m);
    // every staged tuple of the bucket belongs to one of its groups
    // (a consistency check: the plan and the reorder agree)
    for (int q = tid; q < size; q += blockDim.x) {
        const int32_t off = ck[q] >> 10;
        if (off < 0 || off >= z - a) {
            atomicOr(sc.fault, FAULT_TUPLE_RUNS);
            ck[q] = 0 | (ck[q] & 1023);  // keep the reads below inside the bucket
        }
    }
    __syncthreads();
    // values and arrival indices into sorted (group, rank) order
    int32_t tv[PPT], ti[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        const int q = tid + u * PT_THREADS;
        if (q < size) {
            const int p = ck[q] & 1023;
            tv[u] = lv[p];
            ti[u] = li[p];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        const int q = tid + u * PT_THREADS;
        if (q < size) {
            lv[q] = tv[u];
            li[q] = ti[u];
        }
    }
    __syncthreads();
    // Per sorted position q: its group, the group's staged start, old ring
    // pointer, sum and count before the batch.  Every load of a kind is
    // issued for all of a thread's positions before any is used (positions
    // past the bucket are clamped onto its last one and not written).
    int32_t gq[PPT], lq[PPT], pq[PPT], cq[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) gq[u] = a + (ck[min(tid + u * PT_THREADS, size - 1)] >> 10);
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        lq[u] = sc.lpre[gq[u]];
        pq[u] = sc.pold[gq[u]];
        cq[u] = sc.pcnt[gq[u]];
    }
    if (out.passes == 0) {
        long long sq0[PPT];
        int32_t oq[PPT];
#pragma unroll
        for (int u = 0; u < PPT; ++u) sq0[u] = st.sum[gq[u]];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {  // the slot rank r overwrites (read whatever r is)
            const int r = min(tid + u * PT_THREADS, size - 1) - (lq[u] - s0);
            oq[u] = old_slot(st.ring + (int64_t)gq[u] * W, pq[u], r, W);
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int q = tid + u * PT_THREADS;
            if (q >= size) continue;
            const int r = q - (lq[u] - s0);
            const int32_t ev = r < W ? oq[u] : lv[q - W];
            ps[q] = (long long)lv[q] - (long long)ev;
        }
        __syncthreads();
        block_incl_scan_ll(ps, size, reinterpret_cast<long long *>(red));
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int q = tid + u * PT_THREADS;
            if (q >= size) continue;
            const int gs = lq[u] - s0;
            const int r = q - gs;
            const long long s = sq0[u] + ps[q] - (gs > 0 ? ps[gs - 1] : 0);
            const int32_t c = (int32_t)min((int64_t)W, (int64_t)cq[u] + r + 1);
            put(out, li[q], s, c);
        }
        return;
    }
    // From scratch: one tuple per thread.  The old slots come from the
    // ring row (the lanes of a wave mostly hold consecutive ranks of one
    // group, so their reads are consecutive), the values from LDS.  (Copying
    // each group's old window to LDS and rescanning with a wave per group
    // measured slower: a light group can hold up to HEAVY_MIN - 1 tuples,
    // and one wave then carries them all.)
#pragma unroll 1
    for (int u = 0; u < PPT; ++u) {
        const int q = tid + u * PT_THREADS;
        if (q >= size) break;
        const int32_t g = gq[u];
        const int gs = lq[u] - s0;
        const int r = q - gs;
        const int32_t *row = st.ring + (int64_t)g * W;
        const int len = r + 1 < W ? W - (r + 1) : 0;  // old slots still in the window
        const int s1 = (int)(((uint32_t)pq[u] + (uint32_t)(r + 1)) % (uint32_t)W);
        const int n1 = min(len, W - s1);
        const int j0 = max(0, r + 1 - W);
        long long first = 0;
        bool same = true;
        for (int pass = 0; pass < out.passes; ++pass) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            sum_run(row + s1, n1, acc);
            sum_run(row, len - n1, acc);
            sum_run(lv + gs + j0, r - j0 + 1, acc);
            const long long v = (long long)((acc[0] + acc[1]) + (acc[2] + acc[3]));
            if (pass == 0) first = v;
            else same = same && v == first;
            __asm__ volatile("" ::: "memory");  // the next pass reads the window again
        }
        if (!same) atomicOr(sc.fault, FAULT_PASSES);
        const int32_t cn = (int32_t)min((int64_t)W, (int64_t)cq[u] + r + 1);
        put(out, li[q], first, cn);
    }
}

// Ranks [r0, r1) of heavy group x (bucket nl + x).  The item stages the
// piece of seq it needs in LDS: positions [xb, W + r1), the old slots
// (first item only) followed by the values, so every window is one
// contiguous LDS range: window(r) = seq[r+1 .. W+r].
__device__ void heavy_item(int x, int c, int nl, int NB, int tiles, const State &st,
                           const Scratch &sc, const PtOut &out, char *smem) {
    const int tid = threadIdx.x;
    int32_t *rs = reinterpret_cast<int32_t *>(smem + T_RS);
    int32_t *rp = reinterpret_cast<int32_t *>(smem + T_RP);
    int *red = reinterpret_cast<int *>(smem + T_RED);
    int32_t *sq = reinterpret_cast<int32_t *>(smem + H_V);
    int32_t *hi = reinterpret_cast<int32_t *>(smem + H_I);
    long long *ps = reinterpret_cast<long long *>(smem + H_PS);
    const int32_t W = st.W;
    const int32_t g = sc.hkey[x];  // (issued before the rows, which it does not wait on)
    RunRows<PT_THREADS> rr;        // in flight while the group's state is read
    runs_load<PT_THREADS>(sc, nl + x, NB, tiles, rr);
    const int32_t kg = sc.k[g], po = sc.pold[g], cnt0 = sc.pcnt[g];
    const int total = runs_store<PT_THREADS>(tiles, rr, rs, rp, red);
    if (total != kg) {
        if (tid == 0) atomicOr(sc.fault, FAULT_TUPLE_RUNS);
        return;
    }
    const int r0 = c * PT_CH, r1 = min(kg, r0 + PT_CH);
    // LDS index j holds seq position xb + j: the first item from seq[0],
    // later ones (r0 >= PT_CH >= W) from the oldest value of rank r0's
    // window.  window(r) = seq[r+1 .. W+r] is then one contiguous LDS range.
    const int xb = r0 == 0 ? 0 : r0 + 1;
    const int Lq = W + r1 - xb;  // <= PT_CH + PT_WMAX
    const int32_t *row = st.ring + (int64_t)g * W;
    {
        // Both candidate loads of every staged position (an old slot and a
        // staged tuple, indexes clamped into range) are issued before any
        // is used; the position's own kind is kept.
        constexpr int SPT = (H_SPAN + PT_THREADS - 1) / PT_THREADS;
        // (the run searches first: a search is a loop, and loads issued
        // before one would be waited on where it starts)
        int32_t so[SPT], si[SPT], sp[SPT];
        int2 se[SPT];
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int xs = xb + min(tid + u * PT_THREADS, Lq - 1);
            const int rank = max(0, min(xs - W, kg - 1));
            const int r = upper_run(rp, tiles, rank);
            sp[u] = rs[r] + (rank - rp[r]);
        }
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int xs = xb + min(tid + u * PT_THREADS, Lq - 1);
            so[u] = old_slot(row, po, xs, W);
            se[u] = sc.sdat[sp[u]];
            si[u] = sc.sidx[sp[u]];
        }
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            keep(so[u]);
            keep(se[u].y);
            keep(si[u]);
        }
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int j = tid + u * PT_THREADS;
            if (j >= Lq) continue;
            const int xs = xb + j;
            if (xs < W) {
                sq[j] = so[u];
            } else {
                sq[j] = se[u].y;
                if (xs - W >= r0) hi[xs - W - r0] = si[u];
            }
        }
    }
    __syncthreads();
    if (out.passes == 0) {
        for (int j = tid; j < Lq; j += blockDim.x) ps[j] = sq[j];
        __syncthreads();
        block_incl_scan_ll(ps, Lq, reinterpret_cast<long long *>(red));
    }
    for (int r = r0 + tid; r < r1; r += blockDim.x) {
        const int e = W + r - xb;  // window(r) = sq[e - W + 1 .. e]
        long long s;
        if (out.passes == 0) {
            s = ps[e] - (e - W >= 0 ? ps[e - W] : 0);
        } else {
            long long first = 0;
            bool same = true;
            for (int pass = 0; pass < out.passes; ++pass) {
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                sum_run(sq + (e - W + 1), W, acc);
                const long long v = (long long)((acc[0] + acc[1]) + (acc[2] + acc[3]));
                if (pass == 0) first = v;
                else same = same && v == first;
                __asm__ volatile("" ::: "memory");  // the next pass reads the window again
            }
            if (!same) atomicOr(sc.fault, FAULT_PASSES);
            s = first;
        }
        put(out, hi[r - r0], s, (int32_t)min((int64_t)W, (int64_t)cnt0 + r + 1));
    }
}

__global__ __launch_bounds__(PT_THREADS) void k_tuples(State st, Scratch sc, int tiles,
                                                       PtOut out) {
    __shared__ __align__(16) char smem[T_BYTES];
    const PlanTotals t = *sc.tot;
    if (t.status) return;  // rejected batch: nothing to report
    const int nl = t.n_light_buckets, nh = t.n_heavy, NB = t.n_buckets;
    if (NB > NB_MAX || nh > NB_MAX || nl + nh != NB) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(sc.fault, FAULT_TUPLE_RUNS);
        return;
    }
    // heavy work items: ceil(k / PT_CH) per heavy group, prefix in hc
    int32_t *hc = reinterpret_cast<int32_t *>(smem + T_HC);
    int *red = reinterpret_cast<int *>(smem + T_RED);
    for (int x = threadIdx.x; x < nh; x += blockDim.x)
        hc[x] = (sc.k[sc.hkey[x]] + PT_CH - 1) / PT_CH;
    __syncthreads();
    block_excl_scan_array(hc, nh, red);
    const int items = nl + hc[nh];
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        if (it < nl) {
            light_item(it, NB, tiles, st, sc, out, smem);
        } else {
            const int h = it - nl;
            const int x = upper_run(hc, nh, h);  // hc strictly increasing
            heavy_item(x, h - hc[x], nl, NB, tiles, st, sc, out, smem);
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_tuples(State st, Scratch sc, int64_t n, PtOut out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int tiles = (int)((n + PASS_TILE - 1) / PASS_TILE);
    const int64_t want = (n + LIGHT_BUDGET - 1) / LIGHT_BUDGET + (n + PT_CH - 1) / PT_CH + 8;
    const int grid = (int)std::min<int64_t>(PT_GRID_MAX, want);
    hipLaunchKernelGGL(k_tuples, dim3(grid), dim3(PT_THREADS), 0, s, st, sc, tiles, out);
    return hipGetLastError();
}

}  // namespace cq
