"""CPU ORACLE (load-balancing techniques) -- TEST INFRASTRUCTURE ONLY.

The six group-to-thread rebalancing techniques of Section 4 (getFirst,
checkAll, probCheck, bestBalance, shift, shiftLocal; Figures alg1-alg6),
written out in plain Python over ordered per-thread group lists, as the CPU
coordinator of Section 3.1 keeps them.  One call is one rebalancing round
after a batch: it reads the batch's tuples per group and returns the
mapping the next batch runs with (the one-iteration delay of Section 3.1
is the caller's: it applies the result to the following batch).

Where the paper leaves a choice open, these readings are taken:
  * initial mapping: thread w owns groups [ceil(w*G/T), ceil((w+1)*G/T)) in
    id order (Section 5.1: equal shares of consecutive ids);
  * tpt[w] is the sum of the batch counts of the groups in w's list;
  * tmax: the largest tpt, smallest thread id on ties; tmin: the smallest
    tpt, smallest id on ties; a chosen group is the first in list order on
    ties;
  * getFirst/checkAll/probCheck/bestBalance append the chosen group to
    tmin's list.  The loop ends when the gap tpt[tmax] - tpt[tmin] is at
    most the threshold, and also when the chosen group holds at least the
    gap (moving it cannot shrink it: the figures' loop would not end), when
    it holds no tuple (except getFirst, which takes the first group as it
    is), when tmin's list is full (max_keys groups), or after G moves;
  * probCheck: limit = pot * tpt[tmax] / (groups of tmax), a real number;
    the tuples of tmax (the batch's tuples whose group tmax owns at that
    moment) are read in arrival order with a running count per group, and
    the group whose count first reaches the limit is the one moved.  A
    fresh read starts at every iteration of the loop;
  * shift: for tmax > tmin every thread in (tmin, tmax] hands the first
    group of its list to the end of the previous thread's list, otherwise
    every thread in [tmax, tmin) hands its last group to the front of the
    next one's list; a thread with no group hands nothing, a full one takes
    nothing, and threads are taken from the tmin end (each hands on a group
    it held before the round).  Rounds go on while the gap exceeds the
    threshold and stop after a round that moved nothing or left the gap no
    smaller, or once G moves were made;
  * shiftLocal: i = 0 .. T-2 in order, loads updated after every move, the
    group at the end of the list is moved whatever its count.
"""
from __future__ import annotations

GETFIRST, CHECKALL, PROBCHECK, BESTBALANCE, SHIFT, SHIFTLOCAL = range(2, 8)
NAMES = {GETFIRST: "getFirst", CHECKALL: "checkAll", PROBCHECK: "probCheck",
         BESTBALANCE: "bestBalance", SHIFT: "shift", SHIFTLOCAL: "shiftLocal"}


def initial_lists(threads: int, groups: int):
    """Section 5.1: consecutive ids, as equal as possible."""
    def first(w):
        return -(-w * groups // threads)
    return [list(range(first(w), first(w + 1))) for w in range(threads)]


def tuples_per_thread(lists, counts):
    """The tpt vector of the figures."""
    return [sum(int(counts[g]) for g in lst) for lst in lists]


def most_loaded(tpt):
    best = 0
    for w in range(1, len(tpt)):
        if tpt[w] > tpt[best]:
            best = w
    return best


def least_loaded(tpt):
    best = 0
    for w in range(1, len(tpt)):
        if tpt[w] < tpt[best]:
            best = w
    return best


def _choose(policy, lst, counts, tpt, tmax, tmin, pot, keys):
    """The group of tmax that the technique moves (None: no candidate)."""
    if policy == GETFIRST:
        return lst[0]
    if policy == CHECKALL:
        # the most frequent group of the thread's tuples
        best = None
        for g in lst:
            if best is None or counts[g] > counts[best]:
                best = g
        return best
    if policy == PROBCHECK:
        # read the tuples of tmax in arrival order; stop when a group has
        # appeared `limit` times
        limit = pot * tpt[tmax] / len(lst)
        mine = set(lst)
        seen = {}
        for key in keys:
            if key in mine:
                seen[key] = seen.get(key, 0) + 1
                if seen[key] >= limit:
                    return key
        return None
    if policy == BESTBALANCE:
        # the group whose move leaves the pair closest to equal
        best, best_d = None, None
        for g in lst:
            d = abs((tpt[tmax] - counts[g]) - (tpt[tmin] + counts[g]))
            if best_d is None or d < best_d:
                best, best_d = g, d
        return best
    raise ValueError(policy)


def _pair_loop(policy, lists, counts, tpt, threshold, pot, max_keys, groups, keys):
    """Figures alg1-alg4: pair the most and least loaded threads and move one
    group between them until the gap is within the threshold."""
    moves = 0
    while moves < groups:
        tmax, tmin = most_loaded(tpt), least_loaded(tpt)
        gap = tpt[tmax] - tpt[tmin]
        if gap <= threshold:
            break
        g = _choose(policy, lists[tmax], counts, tpt, tmax, tmin, pot, keys)
        if g is None:
            break
        c = counts[g]
        if c >= gap or (c == 0 and policy != GETFIRST) or len(lists[tmin]) >= max_keys:
            break
        lists[tmax].remove(g)
        lists[tmin].append(g)
        tpt[tmax] -= c
        tpt[tmin] += c
        moves += 1
    return moves


def _shift(lists, counts, tpt, threshold, max_keys, groups):
    """Figure alg5: groups travel one neighbour at a time, towards tmin."""
    moves = 0
    while moves < groups:
        tmax, tmin = most_loaded(tpt), least_loaded(tpt)
        gap = tpt[tmax] - tpt[tmin]
        if gap <= threshold:
            break
        before = moves
        if tmax > tmin:
            for i in range(tmin + 1, tmax + 1):
                if lists[i] and len(lists[i - 1]) < max_keys:
                    g = lists[i].pop(0)
                    lists[i - 1].append(g)
                    tpt[i] -= counts[g]
                    tpt[i - 1] += counts[g]
                    moves += 1
        else:
            for i in range(tmin - 1, tmax - 1, -1):
                if lists[i] and len(lists[i + 1]) < max_keys:
                    g = lists[i].pop()
                    lists[i + 1].insert(0, g)
                    tpt[i] -= counts[g]
                    tpt[i + 1] += counts[g]
                    moves += 1
        if moves == before or max(tpt) - min(tpt) >= gap:
            break
    return moves


def _shift_local(lists, counts, tpt, threshold, max_keys):
    """Figure alg6: one pass over neighbouring pairs, no heaps."""
    moves = 0
    for i in range(len(lists) - 1):
        if tpt[i] - tpt[i + 1] > threshold:
            if lists[i] and len(lists[i + 1]) < max_keys:
                g = lists[i].pop()
                lists[i + 1].insert(0, g)
                tpt[i] -= counts[g]
                tpt[i + 1] += counts[g]
                moves += 1
        elif tpt[i + 1] - tpt[i] > threshold:
            if lists[i + 1] and len(lists[i]) < max_keys:
                g = lists[i + 1].pop(0)
                lists[i].append(g)
                tpt[i + 1] -= counts[g]
                tpt[i] += counts[g]
                moves += 1
    return moves


def rebalance(policy, lists, counts, threshold=1000, pot=0.5, max_keys=2048, keys=None):
    """One round of technique ``policy`` on ``lists`` (modified in place) for
    a batch with ``counts[g]`` tuples of group g; returns the moves made.
    ``keys`` are the batch's group ids in arrival order, which probCheck
    reads (the others need only the counts)."""
    counts = [int(c) for c in counts]
    if policy == PROBCHECK:
        if keys is None:
            raise ValueError("probCheck reads the batch's tuples: pass keys")
        keys = [int(k) for k in keys]
    groups = sum(len(lst) for lst in lists)
    tpt = tuples_per_thread(lists, counts)
    if policy == SHIFTLOCAL:
        return _shift_local(lists, counts, tpt, threshold, max_keys)
    if policy == SHIFT:
        return _shift(lists, counts, tpt, threshold, max_keys, groups)
    return _pair_loop(policy, lists, counts, tpt, threshold, pot, max_keys, groups, keys)


def to_csr(lists):
    """(wstart, wlist) of a list mapping."""
    wstart, wlist = [0], []
    for lst in lists:
        wlist.extend(lst)
        wstart.append(len(wlist))
    return wstart, wlist


def from_csr(wstart, wlist):
    return [list(wlist[wstart[w]:wstart[w + 1]]) for w in range(len(wstart) - 1)]
