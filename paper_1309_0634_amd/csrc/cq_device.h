// Device helpers shared by the HIP sources: wave and block scans, run
// tables of the reordered tiles, phase clocks.  Internal; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "cq_internal.h"

namespace cq {

// ------------------------------------------------------------ utilities --

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (lane_id() == 0) ? 0ull : (~0ull >> (64 - lane_id()));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Inclusive prefix sum over the 64 lanes of a wave with DPP row shifts and
// row broadcasts (GFX9 cross-lane data movement), without LDS traffic: four
// shifted adds give prefixes inside each row of 16 lanes, two broadcasts
// carry row totals forward.  Lanes with no source add 0.
__device__ __forceinline__ int wave_incl_add(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// One step of wave_incl_add64: both halves of the source lane's partial sum
// moved by the DPP control, added as one 64-bit value.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ long long dpp_add64(long long x) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)((uint64_t)x >> 32), CTRL,
                                               ROW_MASK, 0xf, false);
    return x + (long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The inclusive prefix sum of wave_incl_add for 64-bit values.
__device__ __forceinline__ long long wave_incl_add64(long long x) {
    x = dpp_add64<0x111, 0xf>(x);  // row_shr:1
    x = dpp_add64<0x112, 0xf>(x);  // row_shr:2
    x = dpp_add64<0x114, 0xf>(x);  // row_shr:4
    x = dpp_add64<0x118, 0xf>(x);  // row_shr:8
    x = dpp_add64<0x142, 0xa>(x);  // row_bcast:15
    x = dpp_add64<0x143, 0xc>(x);  // row_bcast:31
    return x;
}

__device__ __forceinline__ int wave_total(int incl) { return __builtin_amdgcn_readlane(incl, 63); }

// Inclusive running maximum over the 64 lanes of non-negative values (the
// same DPP pattern as wave_incl_add; lanes with no source take 0).
__device__ __forceinline__ int wave_incl_max(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
    return x;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive block scan of F ints per thread; `lds` holds F * waves ints.
// Returns the block totals in `total`.  Barriers inside: call uniformly.
template <int F>
__device__ void block_excl_scan(int (&v)[F], int (&total)[F], int *lds) {
    const int lane = lane_id(), wid = threadIdx.x >> 6;
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

// Exclusive scan of a[0, m) in LDS (in place), a[m] = total.  Each thread
// scans a contiguous piece.  Barriers inside.
__device__ void block_excl_scan_array(int32_t *a, int m, int *lds) {
    const int per = (m + blockDim.x - 1) / blockDim.x;
    const int b0 = min(m, (int)threadIdx.x * per), b1 = min(m, b0 + per);
    int f[1] = {0}, t[1];
    for (int i = b0; i < b1; ++i) f[0] += a[i];
    block_excl_scan<1>(f, t, lds);
    for (int i = b0; i < b1; ++i) {
        const int x = a[i];
        a[i] = f[0];
        f[0] += x;
    }
    if (threadIdx.x == 0) a[m] = t[0];
    __syncthreads();
}

__device__ long long block_sum_ll(long long v, long long *lds) {
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum_ll(v);
    if (lane_id() == 0) lds[wid] = v;
    __syncthreads();
    long long t = 0;
    for (int w = 0; w < nw; ++w) t += lds[w];
    __syncthreads();
    return t;
}

// A key as the query sees it: the raw key, or, when the query reduces keys
// (m != 0), the unsigned value of the raw key mod G, without a division:
// for M = floor((2^64 - 1) / G) + 1, a mod G is the high 64 bits of
// (M * a mod 2^64) * G for every 32-bit a (Lemire, Kaser and Kurz, "Faster
// remainder by direct computation", 2019).  G = 1 uses M = 1.
__device__ __forceinline__ int32_t view_key(int32_t raw, uint64_t m, int64_t G) {
    if (!m) return raw;
    const uint64_t low = m * (uint64_t)(uint32_t)raw;
    return (int32_t)__umul64hi(low, (uint64_t)G);
}

// Marks a loaded value as used here, so that the compiler keeps its load
// where it was issued (beside the others) rather than sinking it into the
// branch that uses it, where it would wait alone.
__device__ __forceinline__ void keep(int32_t &x) { __asm__ volatile("" : "+v"(x)); }
__device__ __forceinline__ void keep(int4 &x) {
    __asm__ volatile("" : "+v"(x.x), "+v"(x.y), "+v"(x.z), "+v"(x.w));
}
__device__ __forceinline__ void keep(int64_t &x) { __asm__ volatile("" : "+v"(x)); }

// The valid lanes whose 6-bit value L (a lane id) equals this lane's: six
// ballots, each lane keeping a ballot or its complement by its own bit of
// L, on the two 32-bit halves (the ballots are wave-uniform, so each step is
// a select and an and per half).
__device__ __forceinline__ uint64_t match_lane_id(bool valid, int L) {
    const uint64_t v = ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int bit = 0; bit < 6; ++bit) {
        const bool on = (L >> bit) & 1;
        const uint64_t bb = ballot(on);
        const uint32_t blo = (uint32_t)bb, bhi = (uint32_t)(bb >> 32);
        lo &= on ? blo : ~blo;
        hi &= on ? bhi : ~bhi;
    }
    return ((uint64_t)hi << 32) | lo;
}

// LDS accesses of other lanes of the wave seen from here on.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes of mask m below this one.
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// A pointer into device memory whose address space the compiler cannot see
// (held in a struct, or read back from LDS), as a global one: its accesses
// are then global instructions rather than generic (flat) ones, which would
// also be counted with the LDS accesses and make every LDS wait wait on them.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *global_ptr(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// Largest r in [0, m) with pre[r] <= p (pre ascending, pre[0] = 0 <= p).
__device__ __forceinline__ int upper_run(const int32_t *pre, int m, int p) {
    int lo = 0, hi = m - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Records the device clock for phase `slot` of this workgroup (thread 0).
__device__ __forceinline__ void phase_mark(const Scratch &sc, int kind, int slot) {
    if (sc.phase && threadIdx.x == 0 && blockIdx.x < PHASE_BLOCKS)
        sc.phase[((int64_t)kind * PHASE_BLOCKS + blockIdx.x) * PHASE_SLOTS + slot] =
            (int64_t)wall_clock64();
}

// The runs of bucket b (one per tile, in tile order = arrival order): rs[t]
// = first staged slot, rp[t] = tuples of the bucket in tiles before t,
// rp[tiles] = bucket size.  runs_load issues this thread's row loads (tiles
// tid + j * NT, clamped into [0, tiles), so that every load is issued
// unconditionally and all are in flight together; the caller may issue its
// own loads beside them), runs_store writes the runs to LDS and scans them
// (barriers inside).
template <int NT>
struct RunRows {
    static constexpr int R = (PASS_TILES_MAX + NT - 1) / NT;
    int32_t s[R], e[R];
};

template <int NT>
__device__ void runs_load(const Scratch &sc, int b, int NB, int tiles, RunRows<NT> &rr) {
#pragma unroll
    for (int j = 0; j < RunRows<NT>::R; ++j) {
        const int t = min((int)threadIdx.x + j * NT, tiles - 1);
        const int32_t *row = sc.rowstart + (int64_t)t * (NB + 1);
        rr.s[j] = row[b];
        rr.e[j] = row[b + 1];
    }
}

template <int NT>
__device__ int runs_store(int tiles, const RunRows<NT> &rr, int32_t *rs, int32_t *rp, int *red) {
#pragma unroll
    for (int j = 0; j < RunRows<NT>::R; ++j) {
        const int t = (int)threadIdx.x + j * NT;
        if (t < tiles) {
            rs[t] = t * PASS_TILE + rr.s[j];
            rp[t] = rr.e[j] - rr.s[j];
        }
    }
    __syncthreads();
    block_excl_scan_array(rp, tiles, red);
    return rp[tiles];
}

// Both steps with nothing between them (NT threads per block).
template <int NT>
__device__ int bucket_runs(const Scratch &sc, int b, int NB, int tiles, int32_t *rs,
                           int32_t *rp, int *red) {
    RunRows<NT> rr;
    runs_load<NT>(sc, b, NB, tiles, rr);
    return runs_store<NT>(tiles, rr, rs, rp, red);
}

}  // namespace cq
