// Host-side group-to-worker balancer: the six load-balancing techniques of
// Section 4 (getFirst, checkAll, probCheck, bestBalance, shift, shiftLocal),
// applied after each batch to that batch's per-worker tuple counts; the new
// mapping takes effect from the next batch (Section 3.1: one iteration of
// delay).  Workers are the static partition's workers (one wave each).
//
// Readings where the paper leaves a choice open:
//  - Every worker keeps an ordered list of groups; initially worker w owns
//    [ceil(w*G/T), ceil((w+1)*G/T)) in id order.  tpt[w] is the batch's
//    tuples of the groups in w's list.
//  - tmax is the most loaded worker and tmin the least loaded one, each the
//    smallest id on ties; a chosen group is the first in list order on ties.
//  - getFirst, checkAll, probCheck and bestBalance move the chosen group of
//    tmax to the tail of tmin's list while tpt[tmax] - tpt[tmin] exceeds the
//    threshold.  The loop stops instead when the chosen group has at least
//    gap = tpt[tmax] - tpt[tmin] tuples (moving it would not shrink the
//    pair's gap, and the loop would never end), when it has none
//    (checkAll, probCheck, bestBalance: nothing to balance with it; getFirst
//    moves empty groups, which is what taking the first group does), when
//    tmin already owns max_keys groups, or after G moves.
//  - probCheck's limit is pot * tpt[tmax] / (groups of tmax), a real
//    number; the technique reads tmax's tuples in arrival order and stops
//    at the first group that has appeared limit times.  That group is the
//    one whose ceil(limit)-th tuple comes earliest in the batch, so the step
//    indexes each group's tuple positions once (a counting sort of the
//    batch's keys) and then compares one position per group of tmax,
//    instead of rereading the tuples at every move.
//  - shift moves the head of each list in (tmin, tmax] to the tail of the
//    list before it, or the tail of each list in [tmax, tmin) to the head of
//    the list after it, so lists stay runs of consecutive ids; a worker with
//    an empty list passes nothing and a full one receives nothing.  The
//    workers are taken from the tmin end, so each passes on a group it held
//    before the round.  Rounds
//    repeat while the gap exceeds the threshold and end after a round that
//    moved nothing or did not shrink the gap, or after G moves.
//  - shiftLocal takes i = 0 .. T-2 in order with tpt updated as it goes and
//    moves whatever group is at the end of the list (no condition on its
//    count), as the technique states.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <set>
#include <utility>
#include <vector>

#include "cq.h"
#include "cq_balance.h"

namespace cq {

namespace {

struct Loads {
    std::vector<int64_t> tpt;
    std::set<std::pair<int64_t, int32_t>> order;  // (load, worker)
    explicit Loads(const std::vector<int64_t> &t) : tpt(t) {
        for (int32_t w = 0; w < (int32_t)t.size(); ++w) order.insert({t[w], w});
    }
    void add(int32_t w, int64_t d) {
        order.erase({tpt[w], w});
        tpt[w] += d;
        order.insert({tpt[w], w});
    }
    int32_t argmin() const { return order.begin()->second; }
    int32_t argmax() const {
        // smallest id among the largest loads
        auto it = std::prev(order.end());
        const int64_t top = it->first;
        return order.lower_bound({top, INT32_MIN})->second;
    }
};

}  // namespace

void Balancer::reset(int32_t workers, int64_t groups) {
    T = workers;
    G = groups;
    lists.assign(T, {});
    owner.assign(G, 0);
    for (int32_t w = 0; w < T; ++w) {
        const int64_t a = (w * G + T - 1) / T, b = ((w + 1) * G + T - 1) / T;
        for (int64_t g = a; g < b; ++g) {
            lists[w].push_back((int32_t)g);
            owner[g] = w;
        }
    }
}

void Balancer::move(int32_t g, int32_t from, int32_t to, bool to_head) {
    auto &src = lists[from];
    if (src.front() == g) src.pop_front();
    else if (src.back() == g) src.pop_back();
    else src.erase(std::find(src.begin(), src.end(), g));
    if (to_head) lists[to].push_front(g);
    else lists[to].push_back(g);
    owner[g] = to;
    ++last_moves;
}

int64_t Balancer::step(int policy, const int32_t *k, const int32_t *keys, int64_t n) {
    std::vector<int64_t> tpt(T, 0);
    for (int32_t w = 0; w < T; ++w)
        for (int32_t g : lists[w]) tpt[w] += k[g];
    last_max = *std::max_element(tpt.begin(), tpt.end());
    last_min = *std::min_element(tpt.begin(), tpt.end());
    last_moves = 0;
    auto room = [&](int32_t w) { return (int64_t)lists[w].size() < max_keys; };
    if (policy == CQ_PARTITION_SHIFTLOCAL) {
        for (int32_t i = 0; i + 1 < T; ++i) {
            if (tpt[i] - tpt[i + 1] > threshold) {
                if (lists[i].empty() || !room(i + 1)) continue;
                const int32_t g = lists[i].back();
                move(g, i, i + 1, true);
                tpt[i] -= k[g];
                tpt[i + 1] += k[g];
            } else if (tpt[i + 1] - tpt[i] > threshold) {
                if (lists[i + 1].empty() || !room(i)) continue;
                const int32_t g = lists[i + 1].front();
                move(g, i + 1, i, false);
                tpt[i + 1] -= k[g];
                tpt[i] += k[g];
            }
        }
        return last_moves;
    }
    // probCheck: the arrival positions of each group's tuples, grouped by
    // group (pstart[g] .. pstart[g+1]) in arrival order
    std::vector<int64_t> pstart, ppos;
    if (policy == CQ_PARTITION_PROBCHECK) {
        pstart.assign(G + 1, 0);
        for (int64_t i = 0; i < n; ++i) ++pstart[keys[i] + 1];
        for (int64_t g = 0; g < G; ++g) pstart[g + 1] += pstart[g];
        ppos.resize(n);
        std::vector<int64_t> fill(pstart.begin(), pstart.end() - 1);
        for (int64_t i = 0; i < n; ++i) ppos[fill[keys[i]]++] = i;
    }
    Loads L(tpt);
    while (last_moves < G) {
        const int32_t tmax = L.argmax(), tmin = L.argmin();
        const int64_t gap = L.tpt[tmax] - L.tpt[tmin];
        if (gap <= threshold) break;
        if (policy == CQ_PARTITION_SHIFT) {
            const int64_t m0 = last_moves;
            if (tmax > tmin) {
                for (int32_t i = tmin + 1; i <= tmax; ++i) {
                    if (lists[i].empty() || !room(i - 1)) continue;
                    const int32_t g = lists[i].front();
                    move(g, i, i - 1, false);
                    L.add(i, -k[g]);
                    L.add(i - 1, k[g]);
                }
            } else {
                for (int32_t i = tmin - 1; i >= tmax; --i) {
                    if (lists[i].empty() || !room(i + 1)) continue;
                    const int32_t g = lists[i].back();
                    move(g, i, i + 1, true);
                    L.add(i, -k[g]);
                    L.add(i + 1, k[g]);
                }
            }
            const int64_t after = L.tpt[L.argmax()] - L.tpt[L.argmin()];
            if (last_moves == m0 || after >= gap) break;
            continue;
        }
        const auto &src = lists[tmax];
        int32_t g = -1;
        if (policy == CQ_PARTITION_GETFIRST) {
            g = src.front();  // tmax is loaded, so its list is not empty
        } else if (policy == CQ_PARTITION_CHECKALL) {
            int64_t best = -1;
            for (int32_t h : src)
                if (k[h] > best) {
                    best = k[h];
                    g = h;
                }
        } else if (policy == CQ_PARTITION_PROBCHECK) {
            // a group "appears limit times" at its ceil(limit)-th tuple; the
            // scan of tmax's tuples stops at the earliest such position
            const double limit = pot * (double)L.tpt[tmax] / (double)src.size();
            const int64_t need = (int64_t)std::ceil(limit);
            int64_t first = INT64_MAX;
            for (int32_t h : src) {
                const int64_t have = pstart[h + 1] - pstart[h];
                if (need < 1 || have < need) continue;
                const int64_t at = ppos[pstart[h] + need - 1];
                if (at < first) {
                    first = at;
                    g = h;
                }
            }
        } else if (policy == CQ_PARTITION_BESTBALANCE) {
            int64_t best = INT64_MAX;
            for (int32_t h : src) {
                const int64_t d = std::llabs((L.tpt[tmax] - k[h]) - (L.tpt[tmin] + k[h]));
                if (d < best) {
                    best = d;
                    g = h;
                }
            }
        } else {
            break;
        }
        if (g < 0) break;
        const int64_t c = k[g];
        if (c >= gap || (c == 0 && policy != CQ_PARTITION_GETFIRST) || !room(tmin)) break;
        move(g, tmax, tmin, false);
        L.add(tmax, -c);
        L.add(tmin, c);
    }
    return last_moves;
}

void Balancer::export_csr(int32_t *wstart, int32_t *wlist, int32_t *lidx) const {
    int32_t p = 0;
    for (int32_t w = 0; w < T; ++w) {
        wstart[w] = p;
        int32_t i = 0;
        for (int32_t g : lists[w]) {
            wlist[p++] = g;
            if (lidx) lidx[g] = i;
            ++i;
        }
    }
    wstart[T] = p;
}

bool Balancer::import_csr(int32_t workers, int64_t groups, const int32_t *wstart,
                          const int32_t *wlist) {
    if (workers < 1 || groups < 1 || wstart[0] != 0 || wstart[workers] != groups) return false;
    std::vector<char> seen(groups, 0);
    T = workers;
    G = groups;
    lists.assign(T, {});
    owner.assign(G, 0);
    for (int32_t w = 0; w < T; ++w) {
        if (wstart[w + 1] < wstart[w]) return false;
        for (int32_t p = wstart[w]; p < wstart[w + 1]; ++p) {
            const int32_t g = wlist[p];
            if (g < 0 || g >= groups || seen[g]) return false;
            seen[g] = 1;
            lists[w].push_back(g);
            owner[g] = w;
        }
    }
    return true;
}

}  // namespace cq

extern "C" int cq_policy_apply(int32_t policy, int32_t workers, int64_t groups,
                               const int32_t *counts, const int32_t *keys, int64_t n,
                               int32_t *wstart, int32_t *wlist, int64_t threshold, double pot,
                               int32_t max_keys, int64_t *moves) {
    if (policy < CQ_PARTITION_GETFIRST || policy > CQ_PARTITION_SHIFTLOCAL) return CQ_ERR_INVALID;
    if (!counts || !wstart || !wlist || !moves || threshold < 0 || !(pot > 0.0 && pot <= 1.0) ||
        max_keys < 1 || workers < 1 || groups < 1 || n < 0 || (n > 0 && !keys))
        return CQ_ERR_INVALID;
    if (policy == CQ_PARTITION_PROBCHECK) {
        // the tuples must be given, and must be the ones counted
        std::vector<int64_t> seen(groups, 0);
        for (int64_t i = 0; i < n; ++i) {
            if (keys[i] < 0 || keys[i] >= groups) return CQ_ERR_INVALID;
            ++seen[keys[i]];
        }
        for (int64_t g = 0; g < groups; ++g)
            if (seen[g] != counts[g]) return CQ_ERR_INVALID;
    }
    cq::Balancer b;
    if (!b.import_csr(workers, groups, wstart, wlist)) return CQ_ERR_INVALID;
    b.threshold = threshold;
    b.pot = pot;
    b.max_keys = max_keys;
    *moves = b.step(policy, counts, keys, n);
    b.export_csr(wstart, wlist, nullptr);
    return CQ_OK;
}
