"""Checks that pin the Section 4 rebalancing techniques to hand-worked cases
and to properties the figures fix, independently of any implementation.

Each ``pin_*`` takes ``rebalance(policy, lists, counts, threshold, pot,
max_keys, keys) -> moves`` (lists modified in place; ``keys`` are the
batch's group ids in arrival order, which probCheck reads), so the same checks run on
the oracle (``oracle.policies``), on the library's host step, and on
deliberately broken copies of the oracle, where at least one must fail.

The worked cases are derived by hand from Figures alg1-alg6 and the text of
Section 4, under the readings stated in ``oracle/policies.py`` (ties to the
smallest id, a move only while it shrinks the pair's gap, shift rounds end
when the gap stops shrinking).
"""
from __future__ import annotations

import numpy as np

GETFIRST, CHECKALL, PROBCHECK, BESTBALANCE, SHIFT, SHIFTLOCAL = range(2, 8)
PAIR_POLICIES = (GETFIRST, CHECKALL, PROBCHECK, BESTBALANCE)
ALL_POLICIES = PAIR_POLICIES + (SHIFT, SHIFTLOCAL)


def _run(rebalance, policy, lists, counts, threshold, pot=0.5, max_keys=2048, keys=None):
    lists = [list(x) for x in lists]
    moves = rebalance(policy, lists, list(counts), threshold, pot, max_keys, keys)
    return lists, moves


def _arrivals(*runs):
    """Batch keys in arrival order from (group, repeat) runs, and the counts
    they imply (one entry per group id up to the largest)."""
    keys = [g for g, r in runs for _ in range(r)]
    counts = [0] * (max(keys) + 1)
    for g in keys:
        counts[g] += 1
    return keys, counts


def pin_getfirst_worked():
    """Figure alg1: the first group of tmax moves while it shrinks the gap."""
    def check(rebalance):
        # tpt = [1500, 0]: group 0 (600) moves; then tpt = [900, 600], gap
        # 300, and the first group of thread 0 is now group 1 (900 >= 300).
        lists, moves = _run(rebalance, GETFIRST, [[0, 1], [2, 3]], [600, 900, 0, 0], 100)
        assert (lists, moves) == ([[1], [2, 3, 0]], 1), (lists, moves)
        # a first group holding the whole gap is not moved
        lists, moves = _run(rebalance, GETFIRST, [[0, 1], [2, 3]], [1500, 10, 5, 5], 1000)
        assert (lists, moves) == ([[0, 1], [2, 3]], 0), (lists, moves)
        # a gap equal to the threshold is not an imbalance
        lists, moves = _run(rebalance, GETFIRST, [[0, 1], [2, 3]], [50, 50, 0, 0], 100)
        assert (lists, moves) == ([[0, 1], [2, 3]], 0), (lists, moves)
        # empty first groups are taken as they come (getFirst does not look)
        lists, moves = _run(rebalance, GETFIRST, [[0, 1, 2], [3]], [0, 0, 700, 0], 100)
        assert (lists, moves) == ([[2], [3, 0, 1]], 2), (lists, moves)
    return check


def pin_checkall_worked():
    """Figure alg2: the most frequent group of tmax moves."""
    def check(rebalance):
        # tpt = [1500, 0]: group 1 (900) moves; tpt = [600, 900]; thread 1's
        # most frequent group is group 1 again, 900 >= gap 300: stop.
        lists, moves = _run(rebalance, CHECKALL, [[0, 1], [2, 3]], [600, 900, 0, 0], 100)
        assert (lists, moves) == ([[0], [2, 3, 1]], 1), (lists, moves)
        # three threads: tpt = [1000, 100, 0]; group 1 (400) to thread 2 ->
        # [600, 100, 400]; group 0 (300) to thread 1 -> [300, 400, 400];
        # gap 100 is not above the threshold 100.
        lists, moves = _run(rebalance, CHECKALL, [[0, 1, 2], [3], [4]],
                            [300, 400, 300, 100, 0], 100)
        assert (lists, moves) == ([[2], [3, 0], [4, 1]], 2), (lists, moves)
    return check


def pin_probcheck_worked():
    """Figure alg3: limit = pot * tpt[tmax] / ngroups; the tuples of tmax are
    read in arrival order and the first group to appear limit times moves."""
    def check(rebalance):
        # tpt = [1000, 0], limit 0.5*1000/4 = 125.  Group 2's first 130
        # tuples arrive first, so it reaches 125 before group 1 (which a
        # scan of the list in id order would take): group 2 (500) moves ->
        # [500, 500], done.
        keys, counts = _arrivals((2, 130), (0, 100), (1, 400), (2, 370))
        counts += [0] * (5 - len(counts))
        lists, moves = _run(rebalance, PROBCHECK, [[0, 1, 2, 3], [4]], counts, 100, pot=0.5,
                            keys=keys)
        assert (lists, moves) == ([[0, 1, 3], [4, 2]], 1), (lists, moves)
        # tpt = [600, 0], limit 0.5*600/3 = 100: group 2 (100 tuples, all
        # arriving first) reaches exactly 100 -> moves: [500, 100]; limit
        # 0.5*500/2 = 125, thread 0's tuples are groups 1 then 0: group 1
        # (300) moves -> [200, 400]; now tmax = 1 with groups [3, 2, 1],
        # limit 0.5*400/3 = 66.7, group 2 arrives first again -> back to
        # thread 0: [300, 300].  (Counts in list order would move group 0
        # first, then stop at group 1 = 300 >= gap 200.)
        keys, counts = _arrivals((2, 100), (1, 300), (0, 200))
        counts += [0] * (4 - len(counts))
        lists, moves = _run(rebalance, PROBCHECK, [[0, 1, 2], [3]], counts, 50, pot=0.5,
                            keys=keys)
        assert (lists, moves) == ([[0, 2], [3, 1]], 3), (lists, moves)
        # pot = 1: the limit is the average (1000/4 = 250): groups 1 and 3
        # arrive first but hold only 200 each; group 2 reaches 250
        keys, counts = _arrivals((1, 200), (3, 200), (2, 500), (0, 100))
        counts += [0] * (5 - len(counts))
        lists, moves = _run(rebalance, PROBCHECK, [[0, 1, 2, 3], [4]], counts, 100, pot=1.0,
                            keys=keys)
        assert (lists, moves) == ([[0, 1, 3], [4, 2]], 1), (lists, moves)
        # only tmax's tuples are read: group 2 (thread 1) arrives first and
        # is skipped; group 1 reaches 0.5*600/2 = 150 and moves to tmin =
        # thread 2 -> [100, 300, 500]; then tmax = 2 (groups 3, 1), limit
        # 125: group 1 again, 500 >= gap 400: stop
        keys, counts = _arrivals((2, 300), (1, 500), (0, 100))
        counts += [0] * (4 - len(counts))
        lists, moves = _run(rebalance, PROBCHECK, [[0, 1], [2], [3]], counts, 50, pot=0.5,
                            keys=keys)
        assert (lists, moves) == ([[0], [2], [3, 1]], 1), (lists, moves)
    return check


def pin_bestbalance_worked():
    """Figure alg4: the group minimising |(tpt[tmax]-c) - (tpt[tmin]+c)|."""
    def check(rebalance):
        # tpt = [1000, 0]: |1000 - 2c| is 0 for group 0 (500): one move
        lists, moves = _run(rebalance, BESTBALANCE, [[0, 1, 2], [3]], [500, 300, 200, 0], 50)
        assert (lists, moves) == ([[1, 2], [3, 0]], 1), (lists, moves)
        # unlike checkAll it does not take the largest group: tpt = [1000, 0]
        # with groups 700, 250, 50 -> 250 leaves |500| vs 700 |400| -> 700
        lists, moves = _run(rebalance, BESTBALANCE, [[0, 1, 2], [3]], [700, 250, 50, 0], 50)
        assert lists[1][1] == 0, (lists, moves)
        lists, moves = _run(rebalance, BESTBALANCE, [[0, 1, 2], [3]], [550, 400, 50, 0], 50)
        # |1000-1100| = 100 (group 0) vs |1000-800| = 200 (group 1): group 0
        assert lists[1][1] == 0, (lists, moves)
        # tmin loaded too: tpt = [1000, 400], gap 600; group 1 (300) evens
        # the pair exactly, the larger group 0 (600) would not shrink the gap
        lists, moves = _run(rebalance, BESTBALANCE, [[0, 1, 2], [3]], [600, 300, 100, 400], 50)
        assert (lists, moves) == ([[0, 2], [3, 1]], 1), (lists, moves)
    return check


def pin_shift_worked():
    """Figure alg5: every thread between tmax and tmin hands one boundary
    group on towards tmin."""
    def check(rebalance):
        # tpt = [0, 0, 800], tmax 2 > tmin 0: group 2 -> thread 0, group 4
        # (700) -> thread 1: [0, 700, 100], gap 700 < 800, go on; tmax 1,
        # tmin 0: group 3 -> thread 0, gap still 700: stop.
        lists, moves = _run(rebalance, SHIFT, [[0, 1], [2, 3], [4, 5]],
                            [0, 0, 0, 0, 700, 100], 100)
        assert (lists, moves) == ([[0, 1, 2, 3], [4], [5]], 3), (lists, moves)
        # tmax 0 < tmin 1: group 1 -> front of thread 1: [300, 300, 0], gap
        # 300 < 600, go on; tmax 0 < tmin 2: thread 1 passes group 3, then
        # thread 0 group 0: [0, 600, 0], gap 600 >= 300: stop (kept).
        lists, moves = _run(rebalance, SHIFT, [[0, 1], [2, 3], [4, 5]],
                            [300, 300, 0, 0, 0, 0], 100)
        assert (lists, moves) == ([[], [0, 1, 2], [3, 4, 5]], 3), (lists, moves)
    return check


def pin_shiftlocal_worked():
    """Figure alg6: one pass over neighbours, last group right or first
    group left."""
    def check(rebalance):
        # i=0: 1200 - 0 > 100 -> group 1 (400) to the front of thread 1;
        # i=1: 400 - 0 > 100 -> group 3 (0 tuples) to the front of thread 2
        lists, moves = _run(rebalance, SHIFTLOCAL, [[0, 1], [2, 3], [4, 5]],
                            [800, 400, 0, 0, 0, 0], 100)
        assert (lists, moves) == ([[0], [1, 2], [3, 4, 5]], 2), (lists, moves)
        # the right neighbour heavier: its first group comes left
        lists, moves = _run(rebalance, SHIFTLOCAL, [[0, 1], [2, 3]], [0, 0, 500, 500], 100)
        assert (lists, moves) == ([[0, 1, 2], [3]], 1), (lists, moves)
        # within the threshold nothing moves
        lists, moves = _run(rebalance, SHIFTLOCAL, [[0], [1]], [100, 0], 100)
        assert moves == 0
    return check


def _zipf_keys(rng, groups, n, s):
    """Batch keys in arrival order (Zipf over permuted ids) and their counts."""
    p = 1.0 / np.arange(1, groups + 1) ** s
    keys = rng.permutation(groups)[rng.choice(groups, size=n, p=p / p.sum())]
    return keys, np.bincount(keys, minlength=groups)


def pin_properties():
    """Properties any step of any technique keeps: the lists stay a partition
    of the groups with at most max_keys each; a pair technique never raises
    the largest load nor lowers the smallest; shift and shiftLocal keep every
    list a run of consecutive ids in thread order."""
    def check(rebalance):
        rng = np.random.default_rng([20130909, 77])
        for trial in range(12):
            T = int(rng.integers(2, 12))
            G = int(rng.integers(T, 60))
            first = [-(-w * G // T) for w in range(T + 1)]
            for policy in ALL_POLICIES:
                lists = [list(range(first[w], first[w + 1])) for w in range(T)]
                for batch in range(4):
                    keys, counts = _zipf_keys(rng, G, int(rng.integers(0, 3000)), 1.2)
                    before = [sum(int(counts[g]) for g in x) for x in lists]
                    cap = max(len(x) for x in lists) + 3
                    moves = rebalance(policy, lists, [int(c) for c in counts], 50, 0.5, cap,
                                      keys)
                    flat = sorted(g for x in lists for g in x)
                    assert flat == list(range(G)), (policy, lists)
                    assert all(len(x) <= cap for x in lists)
                    assert moves >= 0
                    after = [sum(int(counts[g]) for g in x) for x in lists]
                    if policy in PAIR_POLICIES:
                        assert max(after) <= max(before) and min(after) >= min(before), \
                            (policy, before, after)
                    if policy in (SHIFT, SHIFTLOCAL):
                        run = [g for x in lists for g in x]
                        assert run == list(range(G)), (policy, lists)
    return check


ALL_PINS = [pin_getfirst_worked, pin_checkall_worked, pin_probcheck_worked,
            pin_bestbalance_worked, pin_shift_worked, pin_shiftlocal_worked, pin_properties]
