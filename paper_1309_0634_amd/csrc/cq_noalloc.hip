// Working memory of cq_push_batch_results_noalloc: one file-scope device
// array per GPU, sized for the largest batch that entry point accepts, so
// that the call itself never allocates.  The array's address on each device
// is looked up once (hipGetSymbolAddress with that device current) and kept;
// host code only ever hands that address to kernels, never the array's name.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cq.h"
#include "cq_internal.h"

namespace cq {

namespace {

constexpr int64_t NA_G = PASS_LOCAL_G;  // groups: the plan runs inside the reorder pass
constexpr int64_t NA_N = CQ_NOALLOC_MAX_BATCH;
constexpr int64_t NA_TILES = NA_N / PASS_TILE;
// buckets of one batch of at most NA_N tuples: light buckets of LIGHT_BUDGET
// tuples plus one per heavy group (at least HEAVY_MIN tuples each)
constexpr int64_t NA_NB = NA_N / LIGHT_BUDGET + NA_N / HEAVY_MIN + 2;
static_assert(NA_N % PASS_TILE == 0, "whole tiles");
static_assert(NA_N <= SUB, "a single sub-batch");
static_assert(NA_NB <= NB_MAX, "within the kernels' bucket limit");

constexpr int64_t al(int64_t b) { return (b + 255) / 256 * 256; }
// byte offsets of the arrays inside the scratch area
constexpr int64_t O_K = 0;                                   // int32[NA_G] histogram
constexpr int64_t O_LPRE = O_K + al(4 * NA_G);               // int32[NA_G + 1]
constexpr int64_t O_BUCKET = O_LPRE + al(4 * (NA_G + 1));    // int32[NA_G]
constexpr int64_t O_POLD = O_BUCKET + al(4 * NA_G);          // int32[NA_G]
constexpr int64_t O_TIDX = O_POLD + al(4 * NA_G);            // int32[NA_G]
constexpr int64_t O_STAMP = O_TIDX + al(4 * NA_G);           // int32[NA_G]
constexpr int64_t O_TOUCHED = O_STAMP + al(4 * NA_G);        // int32[NA_G]
constexpr int64_t O_NCNT = O_TOUCHED + al(4 * NA_G);         // int32[NA_G]
constexpr int64_t O_BSTART = O_NCNT + al(4 * NA_G);          // int32[NA_NB + 1]
constexpr int64_t O_HKEY = O_BSTART + al(4 * (NA_NB + 1));   // int32[NA_NB]
constexpr int64_t O_SDAT = O_HKEY + al(4 * NA_NB);           // int2[NA_N]
constexpr int64_t O_ROWS = O_SDAT + al(8 * NA_N);            // int32[NA_TILES][NA_NB + 1]
constexpr int64_t O_PART = O_ROWS + al(4 * NA_TILES * (NA_NB + 1));
constexpr int64_t O_TOT = O_PART + al(4 * PLAN_FIELDS * ((NA_G + PLAN_CHUNK - 1) / PLAN_CHUNK));
constexpr int64_t O_BAD = O_TOT + al(sizeof(PlanTotals));
constexpr int64_t NA_BYTES = O_BAD + al(4);
static_assert(NA_BYTES <= CQ_NOALLOC_SCRATCH_BYTES, "the scratch area holds every array");

// The working memory.  Each GPU the library runs on holds its own copy
// until the process ends; every call on that GPU shares it.
static __device__ __align__(256) char scratch[CQ_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
char *g_ptr[MAX_DEVICES] = {};  // device address of `scratch`, per device

// Clears what the next batch needs zeroed: the histogram counters the
// in-pass plan reads (NA_G of them, whatever the query's group count) and
// the bad-key flag.  A plain kernel, not a memset, so that the call can be
// captured into a graph.
__global__ void k_noalloc_clear(int32_t *k, int32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NA_G) k[i] = 0;
    if (i == 0) *bad = 0;
}

}  // namespace

// The scratch area's address on `device` (which must be current), looked
// up at the first call on that device; nullptr if the lookup failed.
char *noalloc_base(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_ptr[device] = static_cast<char *>(p);
    }
    return g_ptr[device];
}

// Batch-local buffers carved out of the scratch area at `base`.
Scratch noalloc_set(char *base) {
    Scratch b{};
    auto at = [&](int64_t off) { return reinterpret_cast<int32_t *>(base + off); };
    b.k = at(O_K);
    b.lpre = at(O_LPRE);
    b.bucket = at(O_BUCKET);
    b.pold = at(O_POLD);
    b.tidx = at(O_TIDX);
    b.stamp = at(O_STAMP);
    b.touched = at(O_TOUCHED);
    b.ncnt = at(O_NCNT);
    b.bstart = at(O_BSTART);
    b.hkey = at(O_HKEY);
    b.sdat = reinterpret_cast<int2 *>(base + O_SDAT);
    b.rowstart = at(O_ROWS);
    b.partials = at(O_PART);
    b.tot = reinterpret_cast<PlanTotals *>(base + O_TOT);
    b.bad = at(O_BAD);
    return b;
}

hipError_t launch_noalloc_clear(const Scratch &sc, hipStream_t s) {
    hipLaunchKernelGGL(k_noalloc_clear, dim3((unsigned)((NA_G + 255) / 256)), dim3(256), 0, s,
                       sc.k, sc.bad);
    return hipGetLastError();
}

}  // namespace cq
