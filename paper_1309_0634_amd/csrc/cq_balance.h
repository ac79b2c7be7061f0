// Host-side balancer of the paper's load-balancing techniques (see
// cq_balance.cpp).  Internal; not part of the ABI.
#pragma once

#include <cstdint>
#include <deque>
#include <vector>

namespace cq {

struct Balancer {
    int32_t T = 0;                           // workers
    int64_t G = 0;                           // groups
    std::vector<std::deque<int32_t>> lists;  // groups of each worker, in order
    std::vector<int32_t> owner;              // worker of each group
    int64_t threshold = 1000;                // imbalance threshold (tuples)
    double pot = 0.5;                        // probCheck's fraction of the average
    int64_t max_keys = 1 << 30;              // most groups one worker may own
    int64_t last_moves = 0;                  // groups moved by the last step
    int64_t last_max = 0, last_min = 0;      // tuples per worker before it

    // Initial mapping: contiguous id ranges of (almost) equal size.
    void reset(int32_t workers, int64_t groups);
    // One balancing step of `policy` (a CQ_PARTITION_* technique) on the
    // batch counts k[G]; probCheck also reads the batch's n group ids in
    // arrival order (keys, each in [0, G)).  Returns the number of groups
    // moved.
    int64_t step(int policy, const int32_t *k, const int32_t *keys = nullptr, int64_t n = 0);
    // Lists as CSR: wstart[T+1], wlist[G]; lidx[g] = position in its list.
    void export_csr(int32_t *wstart, int32_t *wlist, int32_t *lidx) const;
    bool import_csr(int32_t workers, int64_t groups, const int32_t *wstart, const int32_t *wlist);

  private:
    void move(int32_t g, int32_t from, int32_t to, bool to_head);
};

}  // namespace cq
