"""Section 4 rebalancing techniques on the host (CPU only).

The oracle (oracle/policies.py) is pinned to hand-worked cases and to
properties (tests/policy_pins.py); the library's own host step
(cq_policy_apply, the step a push runs after each batch under a technique)
must then return exactly the oracle's mapping, round after round, on seeded
Zipf batches of the paper's shapes."""
import numpy as np
import pytest

import paper_1309_0634_amd as cq
import policy_pins as P
from oracle import policies as O


@pytest.fixture(scope="module")
def L():
    try:
        return cq.lib()
    except ImportError:
        import __graft_entry__
        __graft_entry__.build()
        return cq.lib()


def lib_rebalance(policy, lists, counts, threshold, pot, max_keys, keys=None):
    """The library's host step, through the C-ABI, on list form."""
    wstart, wlist = O.to_csr(lists)
    ws = np.asarray(wstart, dtype=np.int32)
    wl = np.asarray(wlist, dtype=np.int32)
    moves = cq.policy_apply(policy, np.asarray(counts, dtype=np.int32), ws, wl,
                            threshold, pot, max_keys,
                            None if keys is None else np.asarray(keys, dtype=np.int32))
    lists[:] = O.from_csr(ws.tolist(), wl.tolist())
    return moves


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda p: p.__name__)
def test_oracle_pins(pin):
    pin()(O.rebalance)


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda p: p.__name__)
def test_library_pins(pin, L):
    pin()(lib_rebalance)


def _zipf_keys(rng, groups, n, s):
    p = 1.0 / np.arange(1, groups + 1, dtype=np.float64) ** s
    return rng.permutation(groups)[rng.choice(groups, size=n, p=p / p.sum())]


# (threads, groups, tuples per batch, zipf s, threshold, max_keys)
CASES = [
    (4, 100, 5000, 1.0, 100, 2048),       # the paper's small grid
    (64, 1000, 50000, 1.5, 1000, 2048),   # 50K-tuple batches (Section 5.1)
    (256, 1000, 50000, 0.5, 1000, 2048),
    (1024, 10000, 200000, 1.5, 1000, 2048),
    (16, 200, 20000, 2.0, 10, 16),        # tight list capacity
    (7, 50, 3000, 0.0, 0, 2048),          # threshold 0, uniform keys
]


@pytest.mark.parametrize("policy", sorted(O.NAMES), ids=lambda p: O.NAMES[p])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"T{c[0]}_G{c[1]}_s{c[3]}")
def test_library_matches_oracle(policy, case, L):
    T, G, n, s, thr, cap = case
    rng = np.random.default_rng([20130909, 4, T, G, policy])
    ref = O.initial_lists(T, G)
    ws = np.asarray(O.to_csr(ref)[0], dtype=np.int32)
    wl = np.asarray(O.to_csr(ref)[1], dtype=np.int32)
    total = 0
    for batch in range(6):
        keys = _zipf_keys(rng, G, n, s).astype(np.int32)
        counts = np.bincount(keys, minlength=G).astype(np.int32)
        want = O.rebalance(policy, ref, counts.tolist(), thr, 0.5, cap, keys.tolist())
        got = cq.policy_apply(policy, counts, ws, wl, thr, 0.5, cap, keys)
        assert got == want, (batch, got, want)
        assert O.from_csr(ws.tolist(), wl.tolist()) == ref, batch
        total += got
    if s >= 1.0 and thr <= 1000 and policy != O.SHIFTLOCAL:
        assert total > 0  # skewed batches leave something to move


def test_policy_apply_rejects_bad_mappings(L):
    counts = np.zeros(4, dtype=np.int32)
    ok_ws = np.array([0, 2, 4], dtype=np.int32)
    for ws, wl in [(np.array([0, 2, 3], np.int32), np.array([0, 1, 2, 3], np.int32)),
                   (np.array([0, 2, 4], np.int32), np.array([0, 1, 1, 3], np.int32)),
                   (np.array([0, 3, 2], np.int32), np.array([0, 1, 2, 3], np.int32)),
                   (ok_ws.copy(), np.array([0, 1, 2, 9], np.int32))]:
        with pytest.raises(cq.CQError):
            cq.policy_apply(cq.PARTITION_GETFIRST, counts, ws, wl)
    wl = np.arange(4, dtype=np.int32)
    for policy, pot in [(cq.PARTITION_STATIC, 0.5), (8, 0.5), (cq.PARTITION_PROBCHECK, 0.0),
                        (cq.PARTITION_PROBCHECK, 1.5)]:
        with pytest.raises(cq.CQError):
            cq.policy_apply(policy, counts, ok_ws.copy(), wl.copy(), pot=pot)


def test_policy_apply_cost_is_modest(L):
    """One step at the paper's largest grid (64 blocks of 256 threads) over
    10000 groups stays a host-side detail next to a batch."""
    import time
    rng = np.random.default_rng([20130909, 5])
    T, G = 16384, 10000
    keys = _zipf_keys(rng, G, 1 << 20, 1.5).astype(np.int32)
    counts = np.bincount(keys, minlength=G).astype(np.int32)
    for policy in sorted(O.NAMES):
        ws = np.asarray(O.to_csr(O.initial_lists(T, G))[0], np.int32)
        wl = np.arange(G, dtype=np.int32)
        t = time.perf_counter()
        cq.policy_apply(policy, counts, ws, wl, keys=keys)
        assert time.perf_counter() - t < 5.0, O.NAMES[policy]


SRC = open(O.__file__).read()

# plausible mistakes, each planted in a private copy of the oracle
POLICY_MUTANTS = {
    "tmax_largest_id_on_ties": ("if tpt[w] > tpt[best]:", "if tpt[w] >= tpt[best]:"),
    "tmin_largest_id_on_ties": ("if tpt[w] < tpt[best]:", "if tpt[w] <= tpt[best]:"),
    "checkall_last_on_ties": ("counts[g] > counts[best]:", "counts[g] >= counts[best]:"),
    "probcheck_limit_over_all_groups": ("limit = pot * tpt[tmax] / len(lst)",
                                        "limit = pot * tpt[tmax] / len(counts)"),
    "probcheck_strict": ("if seen[key] >= limit:", "if seen[key] > limit:"),
    "probcheck_list_order": ("""        mine = set(lst)
        seen = {}
        for key in keys:
            if key in mine:
                seen[key] = seen.get(key, 0) + 1
                if seen[key] >= limit:
                    return key
        return None""", """        for g in lst:
            if counts[g] >= limit:
                return g
        return None"""),
    "probcheck_reads_every_tuple": ("            if key in mine:\n", "            if True:\n"),
    "bestbalance_one_sided": ("d = abs((tpt[tmax] - counts[g]) - (tpt[tmin] + counts[g]))",
                              "d = abs(tpt[tmax] - tpt[tmin] - counts[g])"),
    "move_equal_to_gap": ("if c >= gap or", "if c > gap or"),
    "threshold_inclusive": ("        if gap <= threshold:\n            break\n        g = _choose",
                            "        if gap < threshold:\n            break\n        g = _choose"),
    "moved_group_to_head": ("lists[tmax].remove(g)\n        lists[tmin].append(g)",
                            "lists[tmax].remove(g)\n        lists[tmin].insert(0, g)"),
    "shift_takes_last_group": ("g = lists[i].pop(0)\n                    lists[i - 1].append(g)",
                               "g = lists[i].pop()\n                    lists[i - 1].append(g)"),
    "shift_stops_late": ("max(tpt) - min(tpt) >= gap", "max(tpt) - min(tpt) > gap"),
    "shiftlocal_first_group_right": ("g = lists[i].pop()\n                lists[i + 1].insert(0, g)",
                                     "g = lists[i].pop(0)\n                lists[i + 1].insert(0, g)"),
}


@pytest.mark.parametrize("name", sorted(POLICY_MUTANTS))
def test_policy_mutant_is_caught(name):
    old, new = POLICY_MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    ns = {"__name__": f"mutant_{name}"}
    exec(compile(SRC.replace(old, new), f"<mutant {name}>", "exec"), ns)
    failed = []
    for pin in P.ALL_PINS:
        try:
            pin()(ns["rebalance"])
        except Exception:  # noqa: BLE001 - any failure counts as caught
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
