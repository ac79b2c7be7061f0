"""Checks that pin the CPU oracle to facts other than its own code.

Each ``pin_*`` function takes a factory ``make(groups, window)`` that returns
an object with ``push(keys, values) -> (ids, sums, counts, avgs)`` and raises
an error carrying ``code == -3`` for a key outside [0, groups).  The checks
are used on the real oracle (``test_oracle_pins.py``) and on deliberately
broken copies of it (``test_oracle_mutants.py``), where at least one check
must fail.

What each pin rests on:
  * brute force: every window rebuilt from the full history (the definition);
  * COUNT closed form: min(W, tuples seen so far by the group);
  * SUM before any eviction: a plain cumulative group-by sum (numpy add.at);
  * W = 1: the value of the group's last tuple in the batch;
  * round-robin keys (the paper's DS1, Section 5.1): arithmetic-series sums;
  * re-interleaving groups (keeping each key's own order) changes nothing;
  * a batch split in two leaves the same state as the whole batch;
  * AVG is the correctly rounded quotient of the exact integers;
  * a bad key rejects the whole batch and changes nothing.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from oracle.brute import BruteForce
from workloads import probe_batch, reinterleave

I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1


def _rng(seed):
    return np.random.default_rng([20130909, seed])


def _as_tuples(res):
    ids, sums, counts, avgs = res
    return [(int(i), int(s), int(c), float(a)) for i, s, c, a in zip(ids, sums, counts, avgs)]


def _same_float(a: float, b: float) -> bool:
    return np.float64(a).tobytes() == np.float64(b).tobytes()


def _assert_equal_results(got, want, ctx=""):
    assert len(got) == len(want), f"{ctx}: {len(got)} vs {len(want)} groups"
    for x, y in zip(got, want):
        assert x[:3] == y[:3], f"{ctx}: {x} vs {y}"
        assert _same_float(x[3], y[3]), f"{ctx}: avg {x[3]!r} vs {y[3]!r}"


def pin_bruteforce(make, cases=40):
    """Ring oracle == brute-force window rebuild, over many wraps."""
    for case in range(cases):
        rng = _rng(case)
        G = int(rng.choice([1, 2, 3, 7, 64]))
        W = int(rng.choice([1, 2, 3, 5, 17, 1000]))
        ora, bf = make(G, W), BruteForce(G, W)
        nb = 12 if W < 1000 else 4
        for b in range(nb):
            n = int(rng.integers(0, 300))
            if case % 5 == 0 and b == 1:
                n = 3 * W + 1 if W < 1000 else 2500   # one batch longer than the window
            keys = rng.integers(0, G, n).astype(np.int32)
            if case % 3 == 0:
                vals = rng.integers(I32_MIN, I32_MAX, n, endpoint=True).astype(np.int32)
            else:
                vals = rng.integers(0, 1_000_000, n).astype(np.int32)
            _assert_equal_results(_as_tuples(ora.push(keys, vals)), bf.push(keys, vals),
                                  f"case {case} G={G} W={W} batch {b}")


def pin_count_closed_form(make):
    """COUNT == min(W, tuples of the group seen so far)."""
    rng = _rng(101)
    G, W = 50, 7
    ora = make(G, W)
    seen = np.zeros(G, np.int64)
    for b in range(20):
        n = int(rng.integers(1, 200))
        keys = rng.integers(0, G, n).astype(np.int32)
        vals = rng.integers(0, 100, n).astype(np.int32)
        np.add.at(seen, keys, 1)
        ids, _, counts, _ = ora.push(keys, vals)
        assert np.array_equal(ids, np.unique(keys))
        assert np.array_equal(counts, np.minimum(W, seen[ids]))


def pin_sum_before_eviction(make):
    """While no group has more than W tuples, SUM is the cumulative
    group-by sum of all tuples so far."""
    rng = _rng(102)
    G, W = 40, 1000
    ora = make(G, W)
    total = np.zeros(G, np.int64)
    seen = np.zeros(G, np.int64)
    for b in range(8):
        keys = rng.integers(0, G, 500).astype(np.int32)
        vals = rng.integers(I32_MIN, I32_MAX, 500, endpoint=True).astype(np.int32)
        np.add.at(total, keys, vals.astype(np.int64))
        np.add.at(seen, keys, 1)
        assert seen.max() <= W
        ids, sums, counts, _ = ora.push(keys, vals)
        assert np.array_equal(sums, total[ids])
        assert np.array_equal(counts, seen[ids])


def pin_w1_last_writer(make):
    """W = 1: SUM is the value of the group's last tuple in the batch."""
    rng = _rng(103)
    G = 30
    ora = make(G, 1)
    for b in range(10):
        n = int(rng.integers(1, 400))
        keys = rng.integers(0, G, n).astype(np.int32)
        vals = rng.integers(I32_MIN, I32_MAX, n, endpoint=True).astype(np.int32)
        rk = keys[::-1]
        uk, first_in_reversed = np.unique(rk, return_index=True)
        last_vals = vals[::-1][first_in_reversed]
        ids, sums, counts, _ = ora.push(keys, vals)
        assert np.array_equal(ids, uk)
        assert np.array_equal(sums, last_vals.astype(np.int64))
        assert np.all(counts == 1)


def _sum_j_mod(x: int, m: int) -> int:
    """sum_{j=0..x} (j mod m) for x >= -1, in closed form."""
    if x < 0:
        return 0
    q, r = divmod(x, m)
    return q * (m * (m - 1) // 2) + r * (r + 1) // 2


def pin_round_robin(make):
    """Round-robin keys (DS1): key_t = t mod G, value_t = t mod M with
    M = G * m.  Group g's window after T tuples holds t = g + jG for the
    last min(W, count) values of j, so its SUM is
    sum_j (g + (j mod m) G) -- an arithmetic series in closed form."""
    for (G, W, m, n, nb) in [(13, 5, 4, 100, 7), (40, 9, 7, 333, 5), (3, 1, 2, 10, 9)]:
        M = G * m
        ora = make(G, W)
        T = 0
        for b in range(nb):
            t = np.arange(T, T + n, dtype=np.int64)
            keys = (t % G).astype(np.int32)
            vals = (t % M).astype(np.int32)
            T += n
            ids, sums, counts, _ = ora.push(keys, vals)
            for g, s, c in zip(ids.tolist(), sums.tolist(), counts.tolist()):
                seen = (T - 1 - g) // G + 1          # tuples t = g + jG < T
                j1 = seen - 1
                j0 = max(0, seen - W)
                cnt = j1 - j0 + 1
                want = cnt * g + G * (_sum_j_mod(j1, m) - _sum_j_mod(j0 - 1, m))
                assert c == min(W, seen)
                assert s == want, (G, W, b, g, s, want)


def pin_reinterleave(make):
    """Re-interleaving groups while keeping each key's own order leaves every
    result unchanged."""
    rng = _rng(104)
    for case in range(6):
        G, W = [(5, 3), (17, 1), (64, 20), (2, 2), (9, 1000), (33, 4)][case]
        a, b = make(G, W), make(G, W)
        for bi in range(6):
            n = int(rng.integers(1, 500))
            keys = rng.integers(0, G, n).astype(np.int32)
            vals = rng.integers(I32_MIN, I32_MAX, n, endpoint=True).astype(np.int32)
            k2, v2 = reinterleave(keys, vals, seed=case * 100 + bi)
            _assert_equal_results(_as_tuples(a.push(keys, vals)), _as_tuples(b.push(k2, v2)),
                                  f"reinterleave case {case}")


def pin_order_matters(make):
    """A full permutation of a batch is NOT neutral once windows evict: with
    W = 1, the batch [(g,5),(g,7)] leaves 7 and the reversed batch leaves 5.
    COUNT is unaffected."""
    a, b = make(1, 1), make(1, 1)
    ra = a.push(np.array([0, 0], np.int32), np.array([5, 7], np.int32))
    rb = b.push(np.array([0, 0], np.int32), np.array([7, 5], np.int32))
    assert int(ra[1][0]) == 7 and int(rb[1][0]) == 5
    assert int(ra[2][0]) == int(rb[2][0]) == 1


def pin_batch_split(make):
    """Pushing B1 then B2 leaves the same windows as pushing B1||B2: the same
    random continuation (and a probe of every group) then gives identical
    results."""
    rng = _rng(105)
    for case in range(5):
        G, W = [(7, 3), (20, 1), (3, 11), (64, 64), (10, 2)][case]
        a, b = make(G, W), make(G, W)
        n = int(rng.integers(2, 400))
        keys = rng.integers(0, G, n).astype(np.int32)
        vals = rng.integers(-1000, 1000, n).astype(np.int32)
        cut = int(rng.integers(1, n))
        a.push(keys, vals)
        b.push(keys[:cut], vals[:cut])
        b.push(keys[cut:], vals[cut:])
        for bi in range(4):
            m = int(rng.integers(1, 100))
            k2 = rng.integers(0, G, m).astype(np.int32)
            v2 = rng.integers(-1000, 1000, m).astype(np.int32)
            _assert_equal_results(_as_tuples(a.push(k2, v2)), _as_tuples(b.push(k2, v2)),
                                  f"split case {case}")
        pk, pv = probe_batch(G)
        for _ in range(W):
            _assert_equal_results(_as_tuples(a.push(pk, pv)), _as_tuples(b.push(pk, pv)),
                                  f"probe case {case}")


def pin_avg_is_rounded_quotient(make):
    """AVG equals the correctly rounded quotient SUM / COUNT of the exact
    integers (checked with exact rationals), including extreme values."""
    rng = _rng(106)
    G, W = 8, 1000
    ora = make(G, W)
    for b in range(6):
        n = 700
        keys = rng.integers(0, G, n).astype(np.int32)
        if b % 2:
            vals = np.where(rng.random(n) < 0.5, I32_MAX, I32_MIN).astype(np.int32)
        else:
            vals = rng.integers(I32_MIN, I32_MAX, n, endpoint=True).astype(np.int32)
        ids, sums, counts, avgs = ora.push(keys, vals)
        for s, c, a in zip(sums.tolist(), counts.tolist(), avgs.tolist()):
            exact = Fraction(s, c)
            # a is the double nearest to exact: its neighbours are no closer
            lo, hi = np.nextafter(a, -np.inf), np.nextafter(a, np.inf)
            assert abs(Fraction(a) - exact) <= abs(Fraction(float(lo)) - exact)
            assert abs(Fraction(a) - exact) <= abs(Fraction(float(hi)) - exact)
            assert _same_float(a, s / c)


def pin_bad_key_rejects(make):
    """A key outside [0, G) rejects the whole batch and changes nothing."""
    rng = _rng(107)
    G, W = 6, 4
    a, b = make(G, W), make(G, W)
    k1 = rng.integers(0, G, 50).astype(np.int32)
    v1 = rng.integers(0, 100, 50).astype(np.int32)
    a.push(k1, v1)
    b.push(k1, v1)
    for bad in (G, -1, 1 << 30):
        kb = rng.integers(0, G, 30).astype(np.int32)
        kb[17] = bad
        try:
            a.push(kb, rng.integers(0, 100, 30).astype(np.int32))
        except Exception as e:  # noqa: BLE001
            assert getattr(e, "code", None) == -3
        else:
            raise AssertionError("bad key accepted")
    for _ in range(5):
        k2 = rng.integers(0, G, 40).astype(np.int32)
        v2 = rng.integers(0, 100, 40).astype(np.int32)
        _assert_equal_results(_as_tuples(a.push(k2, v2)), _as_tuples(b.push(k2, v2)), "after reject")


def pin_empty_batch(make):
    """An empty batch touches nothing and changes nothing."""
    a, b = make(5, 3), make(5, 3)
    k = np.array([1, 1, 2, 4, 1], np.int32)
    v = np.array([3, 4, 5, 6, 7], np.int32)
    a.push(k, v)
    b.push(k, v)
    e = np.zeros(0, np.int32)
    assert len(a.push(e, e)[0]) == 0
    _assert_equal_results(_as_tuples(a.push(k, v)), _as_tuples(b.push(k, v)), "after empty")


# ---- per-tuple results (the Section 5.1 aggregate after every insertion) --

def _tuples(res):
    s, c, a = res
    return [(int(x), int(y), float(z)) for x, y, z in zip(s, c, a)]


def pin_tuples_bruteforce(make, cases=30):
    """Per-tuple SUM/COUNT/AVG == the brute-force history slice after each
    tuple, over windows that wrap within and across batches."""
    for case in range(cases):
        rng = _rng(300 + case)
        G = int(rng.integers(1, 9))
        W = int(rng.choice([1, 2, 3, 5, 8, 13]))
        ora, bf = make(G, W), BruteForce(G, W)
        for b in range(int(rng.integers(1, 6))):
            n = int(rng.integers(0, 60))
            keys = rng.integers(0, G, n).astype(np.int32)
            vals = rng.integers(-50, 50, n).astype(np.int32)
            got = _tuples(ora.push_tuples(keys, vals))
            want = bf.push_tuples(keys, vals)
            assert len(got) == len(want)
            for x, y in zip(got, want):
                assert x[:2] == y[:2] and _same_float(x[2], y[2]), (case, b, x, y)


def pin_tuples_last_is_batch_result(make):
    """A group's per-tuple result at its last tuple of the batch is the
    batch's result for that group (per-batch and per-tuple forms agree)."""
    rng = _rng(320)
    for G, W in [(7, 4), (50, 30), (3, 200)]:
        a, b = make(G, W), make(G, W)
        for _ in range(5):
            n = int(rng.integers(1, 400))
            keys = rng.integers(0, G, n).astype(np.int32)
            vals = rng.integers(I32_MIN, I32_MAX, n, endpoint=True).astype(np.int32)
            per = _tuples(a.push_tuples(keys, vals))
            batch = _as_tuples(b.push(keys, vals))
            last = {}
            for i, k in enumerate(keys.tolist()):
                last[k] = i
            assert sorted(last) == [t[0] for t in batch]
            for g, s, c, avg in batch:
                x = per[last[g]]
                assert x[:2] == (s, c) and _same_float(x[2], avg), (G, W, g, x)


def pin_tuples_w1(make):
    """W = 1: every tuple's window is the tuple itself."""
    rng = _rng(321)
    ora = make(9, 1)
    for _ in range(4):
        keys = rng.integers(0, 9, 300).astype(np.int32)
        vals = rng.integers(I32_MIN, I32_MAX, 300, endpoint=True).astype(np.int32)
        s, c, a = ora.push_tuples(keys, vals)
        assert np.array_equal(s, vals.astype(np.int64)) and np.all(c == 1)
        assert np.array_equal(a, vals.astype(np.float64))


def pin_tuples_running_sum(make):
    """With W above every group's tuple count, a tuple's SUM is its group's
    running sum so far and COUNT its running count (numpy cumsum per key)."""
    rng = _rng(322)
    G, W = 6, 1000
    ora = make(G, W)
    hist_s = np.zeros(G, np.int64)
    hist_c = np.zeros(G, np.int64)
    for _ in range(3):
        n = 250
        keys = rng.integers(0, G, n).astype(np.int32)
        vals = rng.integers(I32_MIN, I32_MAX, n, endpoint=True).astype(np.int32)
        s, c, _ = ora.push_tuples(keys, vals)
        for g in range(G):
            m = keys == g
            want = hist_s[g] + np.cumsum(vals[m].astype(np.int64))
            assert np.array_equal(s[m], want)
            assert np.array_equal(c[m], hist_c[g] + np.arange(1, m.sum() + 1))
            if m.any():
                hist_s[g] = want[-1]
                hist_c[g] += m.sum()


def pin_tuples_round_robin(make):
    """Round-robin keys (DS1), value = arrival number t: the tuple t of group
    g = t mod G ends a window of m = min(W, t // G + 1) values t, t-G, ...,
    whose SUM is m*t - G*m*(m-1)/2."""
    for G, W, n, nb in [(5, 3, 97, 4), (16, 40, 1000, 3)]:
        ora = make(G, W)
        T = 0
        for _ in range(nb):
            t = np.arange(T, T + n, dtype=np.int64)
            s, c, _ = ora.push_tuples((t % G).astype(np.int32), t.astype(np.int32))
            m = np.minimum(W, t // G + 1)
            assert np.array_equal(c, m)
            assert np.array_equal(s, m * t - G * m * (m - 1) // 2)
            T += n


def pin_tuples_batch_split(make):
    """Per-tuple results do not depend on where the stream is cut into
    batches: B1||B2 gives the concatenation of B1's and then B2's."""
    rng = _rng(323)
    G, W = 11, 6
    a, b = make(G, W), make(G, W)
    keys = rng.integers(0, G, 500).astype(np.int32)
    vals = rng.integers(-1000, 1000, 500).astype(np.int32)
    whole = _tuples(a.push_tuples(keys, vals))
    cut = int(rng.integers(1, 499))
    parts = _tuples(b.push_tuples(keys[:cut], vals[:cut])) + \
        _tuples(b.push_tuples(keys[cut:], vals[cut:]))
    assert whole == parts


def pin_tuples_bad_key(make):
    """A bad key rejects the batch: no state change (later results equal
    those of a twin that never saw it)."""
    rng = _rng(324)
    a, b = make(5, 4), make(5, 4)
    keys = rng.integers(0, 5, 40).astype(np.int32)
    vals = rng.integers(0, 9, 40).astype(np.int32)
    a.push_tuples(keys, vals)
    b.push_tuples(keys, vals)
    bad = keys.copy()
    bad[7] = 5
    try:
        a.push_tuples(bad, vals)
    except Exception as e:  # noqa: BLE001 - the oracle's own error type
        assert getattr(e, "code", None) == -3
    else:
        raise AssertionError("bad key accepted")
    assert _tuples(a.push_tuples(keys, vals)) == _tuples(b.push_tuples(keys, vals))


ALL_PINS = [pin_bruteforce, pin_count_closed_form, pin_sum_before_eviction,
            pin_w1_last_writer, pin_round_robin, pin_reinterleave, pin_order_matters,
            pin_batch_split, pin_avg_is_rounded_quotient, pin_bad_key_rejects,
            pin_empty_batch, pin_tuples_bruteforce, pin_tuples_last_is_batch_result,
            pin_tuples_w1, pin_tuples_running_sum, pin_tuples_round_robin,
            pin_tuples_batch_split, pin_tuples_bad_key]
