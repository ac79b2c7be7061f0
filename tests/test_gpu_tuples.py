"""GPU parity of the per-tuple variant (cq_push_batch_tuples): for every
tuple, its group's window SUM / COUNT / AVG right after it entered, as the
paper recomputes after each insertion (Section 5.1) -- incrementally
(passes = 0) or summed from scratch 1 or 10 times.  Compared bit for bit
with the CPU oracle's per-tuple form, every tuple."""
import numpy as np
import pytest

import paper_1309_0634_amd as cq
from gpu_helpers import assert_same, device, note, to_dev
from oracle import OracleError, RingOracle
from workloads import host_batch, skew, tiny

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cq.lib()
    torch.cuda.set_device(0)


def check_tuples(q, o, keys, values, passes, ctx):
    """Push through the GPU per-tuple path and the oracle; compare every
    tuple, then the batch's per-group results against the oracle's
    per-tuple results at each group's last tuple."""
    got = q.push_tuples(to_dev(keys), to_dev(values), passes)
    gs, gc, ga = (t.cpu().numpy() for t in got)
    ws, wc, wa = o.push_tuples(keys, values)
    n = len(keys)
    for name, g, w in (("sums", gs, ws), ("counts", gc, wc)):
        if not np.array_equal(g, w):
            i = int(np.flatnonzero(g != w)[0])
            raise AssertionError(f"{ctx}: per-tuple {name} differ at {np.sum(g != w)} of {n}; "
                                 f"first at tuple {i} (group {keys[i]}): gpu {g[i]} oracle {w[i]}")
    assert np.array_equal(ga.view(np.int64), wa.view(np.int64)), f"{ctx}: per-tuple avgs differ"
    last = {}
    for i, k in enumerate(keys.tolist()):
        last[k] = i
    ids = np.array(sorted(last), dtype=np.int32)
    li = np.array([last[g] for g in ids.tolist()], dtype=np.int64)
    want = (ids, ws[li], wc[li], wa[li]) if n else (ids, ws[:0], wc[:0], wa[:0])
    assert_same(q.results(), want, f"{ctx}: batch results")


@pytest.mark.parametrize("passes", [0, 1, 10])
def test_tiny_stream_per_tuple(passes):
    note(f"case: tiny stream per tuple, passes {passes}")
    cfg = tiny()
    q = cq.Query(cfg.groups, cfg.window)
    o = RingOracle(cfg.groups, cfg.window)
    for b in range(12):
        k, v = host_batch(cfg, b)
        check_tuples(q, o, k, v, passes, f"tiny batch {b}")
    q.close()
    o.close()


@pytest.mark.parametrize("W", [1, 2, 3, 7, 100, 1000, 1024])
@pytest.mark.parametrize("passes", [0, 1])
def test_windows_and_heavy_chunks(W, passes):
    """Light groups with k >= W (small W), heavy groups over one, two and
    three rank chunks, windows that wrap inside a batch."""
    note(f"case: per tuple W={W} passes {passes}")
    rng = np.random.default_rng([20130909, 61, W, passes])
    G = 37
    q = cq.Query(G, W)
    o = RingOracle(G, W)
    for b, n in enumerate([1, 300, 4096, 2500, 9000, 70000, 5]):
        k = rng.integers(0, G, n).astype(np.int32)
        if n > 1000:  # hot groups: one over 2048 tuples, one over 1024
            k[rng.random(n) < 0.4] = 3
            k[rng.random(n) < 0.15] = 30
        v = rng.integers(-(1 << 31), (1 << 31) - 1, n, endpoint=True).astype(np.int32)
        check_tuples(q, o, k, v, passes, f"W={W} batch {b} n={n}")
    q.close()
    o.close()


@pytest.mark.parametrize("passes,batches", [(0, 3), (1, 1), (10, 1)])
def test_skew_full_size_per_tuple(passes, batches):
    """10,000 groups, W=1000, 1,048,576-tuple Zipf s=1.5 batches (the hot
    group holds ~38% of a batch)."""
    note(f"case: skew s=1.5 per tuple, passes {passes}")
    cfg = skew(1.5)
    q = cq.Query(cfg.groups, cfg.window)
    o = RingOracle(cfg.groups, cfg.window)
    for b in range(batches + 1):
        k, v = host_batch(cfg, b)
        if b < 1 and batches == 1:  # fill the windows first
            q.push(to_dev(k), to_dev(v))
            o.push(k, v)
            continue
        check_tuples(q, o, k, v, passes, f"skew batch {b}")
    assert q.batch_plan()["fault"] == 0
    q.close()
    o.close()


@pytest.mark.parametrize("passes", [0, 2])
def test_batch_longer_than_a_sub_batch(passes):
    note(f"case: per tuple over two sub-batches, passes {passes}")
    rng = np.random.default_rng([20130909, 62, passes])
    G, W = 300, 50
    q = cq.Query(G, W)
    o = RingOracle(G, W)
    n = (1 << 20) + 5000
    k = np.minimum(rng.zipf(1.3, n) - 1, G - 1).astype(np.int32)
    v = rng.integers(-1000, 1000, n).astype(np.int32)
    check_tuples(q, o, k, v, passes, "two sub-batches")
    k2, v2 = k[:7777].copy(), v[:7777].copy()
    check_tuples(q, o, k2, v2, passes, "after")
    q.close()
    o.close()


def test_rejected_batch_and_mixing_with_plain_pushes():
    note("case: per tuple rejected batch, mixed calls")
    import torch
    rng = np.random.default_rng([20130909, 63])
    G, W = 64, 20
    q = cq.Query(G, W)
    o = RingOracle(G, W)
    for b in range(6):
        n = int(rng.integers(1, 3000))
        k = rng.integers(0, G, n).astype(np.int32)
        v = rng.integers(-99, 99, n).astype(np.int32)
        if b == 2:
            bad = k.copy()
            bad[n // 2] = G
            s = torch.full((n,), 7, dtype=torch.int64, device=device())
            q.push_tuples_into(to_dev(bad), to_dev(v), s, None, None, 0)
            assert q.status() == cq.ERR_KEY_RANGE
            assert bool((s.cpu() == 7).all())
            with pytest.raises(OracleError):
                o.push_tuples(bad, v)
        if b % 2:
            q.push(to_dev(k), to_dev(v))
            assert_same(q.results(), o.push(k, v), f"plain batch {b}")
        else:
            check_tuples(q, o, k, v, b % 3, f"per-tuple batch {b}")
    check_tuples(q, o, np.zeros(0, np.int32), np.zeros(0, np.int32), 0, "empty")
    q.close()
    o.close()


def test_per_tuple_limits():
    note("case: per tuple limits")
    k = to_dev(np.zeros(4, np.int32))
    v = to_dev(np.ones(4, np.int32))
    q = cq.Query(100, cq.TUPLE_MAX_WINDOW + 1)
    with pytest.raises(cq.CQError):
        q.push_tuples(k, v)
    q.close()
    q = cq.Query(cq.TUPLE_MAX_GROUPS + 1, 10)
    with pytest.raises(cq.CQError):
        q.push_tuples(k, v)
    q.close()
    q = cq.Query(100, 10, partition=cq.PARTITION_STATIC)
    with pytest.raises(cq.CQError):
        q.push_tuples(k, v)
    q.set_partition(cq.PARTITION_BALANCED)
    for bad in (-1, cq.TUPLE_MAX_PASSES + 1):
        with pytest.raises(cq.CQError):
            q.push_tuples(k, v, bad)
    s, c, _ = q.push_tuples(k, v, cq.TUPLE_MAX_PASSES)
    assert s.cpu().tolist() == [1, 2, 3, 4] and c.cpu().tolist() == [1, 2, 3, 4]
    q.close()
