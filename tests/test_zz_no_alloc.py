"""The allocation-free entry point (cq_push_batch_results_noalloc) against
cq_push_batch_results on twin queries: same batches, same results bit for
bit, call after call (its working memory is one shared area per GPU that
keeps the previous call's contents), plus its limits."""
import numpy as np
import pytest

import paper_1309_0634_amd as cq
from gpu_helpers import device, note, to_dev
from oracle import RingOracle
from workloads import host_batch, skew

pytestmark = pytest.mark.gpu


def _outs(cap):
    import torch
    dev = device()
    return (torch.empty(cap, dtype=torch.int32, device=dev),
            torch.empty(cap, dtype=torch.int64, device=dev),
            torch.empty(cap, dtype=torch.int32, device=dev),
            torch.empty(cap, dtype=torch.float64, device=dev),
            torch.empty(1, dtype=torch.int64, device=dev))


def _host(outs):
    import torch
    torch.cuda.synchronize()
    m = int(outs[4].cpu().item())
    if m < 0:
        return m, None
    return m, tuple(t[:m].cpu().numpy() for t in outs[:4])


def _same(a, b, ctx):
    ma, ra = a
    mb, rb = b
    assert ma == mb, f"{ctx}: n_touched {ma} vs {mb}"
    if ra is None:
        return
    for x, y, name in zip(ra, rb, ("ids", "sums", "counts", "avgs")):
        if x.dtype == np.float64:
            x, y = x.view(np.int64), y.view(np.int64)
        assert np.array_equal(x, y), f"{ctx}: {name} differs"


def _step(qa, qb, keys, values, ctx, ora=None):
    """One batch through the allocation-free call (qa) and the ordinary one
    (qb); both results, and the oracle's when given, must agree."""
    note(ctx)
    cap = max(1, min(qa.groups, len(keys)))
    oa, ob = _outs(cap), _outs(cap)
    dk, dv = to_dev(keys), to_dev(values)
    qa.push_results_noalloc_into(dk, dv, *oa)
    qb.push_results_into(dk, dv, *ob)
    ra, rb = _host(oa), _host(ob)
    _same(ra, rb, ctx)
    if ora is not None:
        want = ora.push(keys, values)
        assert ra[0] == len(want[0]), f"{ctx}: {ra[0]} touched vs oracle {len(want[0])}"
        _same(ra, (len(want[0]), tuple(np.asarray(w) for w in want)), ctx + " vs oracle")
    return ra


def test_noalloc_equals_push_results_on_consecutive_calls():
    cfg = skew(1.5)
    qa, qb = cq.Query(cfg.groups, cfg.window), cq.Query(cfg.groups, cfg.window)
    ora = RingOracle(cfg.groups, cfg.window)
    try:
        # the largest batch the call takes, then smaller ragged ones
        for b, n in enumerate((cq.NOALLOC_MAX_BATCH, 100_003, 777, cq.NOALLOC_MAX_BATCH - 1)):
            k, v = host_batch(cfg, b, n)
            _step(qa, qb, k, v, f"noalloc skew s=1.5 call {b} n={n}", ora)
    finally:
        qa.close(), qb.close(), ora.close()


def test_noalloc_rejected_batch_then_accepted():
    G, W = 1000, 37
    qa, qb = cq.Query(G, W), cq.Query(G, W)
    ora = RingOracle(G, W)
    rng = np.random.default_rng(5)
    try:
        k = rng.integers(0, G, 5000).astype(np.int32)
        v = rng.integers(0, 10 ** 6, 5000).astype(np.int32)
        _step(qa, qb, k, v, "noalloc first batch", ora)
        kb = k.copy()
        kb[4321] = G  # out of range: the whole batch is rejected
        m, _ = _step(qa, qb, kb, v, "noalloc rejected batch")
        assert m == cq.ERR_KEY_RANGE
        # the bad-key flag the rejection left must not reject the next call
        k2 = rng.integers(0, G, 3000).astype(np.int32)
        v2 = rng.integers(0, 10 ** 6, 3000).astype(np.int32)
        _step(qa, qb, k2, v2, "noalloc batch after a rejection", ora)
    finally:
        qa.close(), qb.close(), ora.close()


def test_noalloc_alternating_queries_share_the_area():
    rng = np.random.default_rng(11)
    shapes = [(64, 1000), (16384, 5), (1, 3), (10000, 1000)]
    pairs = [(cq.Query(G, W), cq.Query(G, W), RingOracle(G, W), G) for G, W in shapes]
    try:
        for rnd in range(3):
            for i, (qa, qb, ora, G) in enumerate(pairs):
                n = int(rng.integers(1, 70_000))
                k = rng.integers(0, G, n).astype(np.int32)
                v = rng.integers(-2 ** 31, 2 ** 31 - 1, n, dtype=np.int64).astype(np.int32)
                _step(qa, qb, k, v, f"noalloc round {rnd} query {i} G={G} n={n}", ora)
    finally:
        for qa, qb, ora, _ in pairs:
            qa.close(), qb.close(), ora.close()


def test_noalloc_key_mod_and_empty_batch():
    G, W = 777, 100
    qa, qb = cq.Query(G, W), cq.Query(G, W)
    qa.set_key_mod(True)
    qb.set_key_mod(True)
    rng = np.random.default_rng(3)
    try:
        k = rng.integers(-2 ** 31, 2 ** 31 - 1, 40_000, dtype=np.int64).astype(np.int32)
        v = rng.integers(0, 10 ** 6, 40_000).astype(np.int32)
        _step(qa, qb, k, v, "noalloc key-mod batch")
        m, _ = _step(qa, qb, k[:0], v[:0], "noalloc empty batch")
        assert m == 0
        _step(qa, qb, k[:1234], v[:1234], "noalloc key-mod batch after an empty one")
    finally:
        qa.close(), qb.close()


def test_noalloc_limits():
    import ctypes
    L = cq.lib()
    import torch
    dev = device()
    note("noalloc limits")
    ok = cq.Query(100, 10)
    big = cq.Query(cq.NOALLOC_MAX_GROUPS + 1, 10)
    stat = cq.Query(100, 10, partition=cq.PARTITION_STATIC)
    try:
        k = torch.zeros(cq.NOALLOC_MAX_BATCH + 1, dtype=torch.int32, device=dev)
        o = _outs(100)
        args = [o[0].data_ptr(), o[1].data_ptr(), o[2].data_ptr(), o[3].data_ptr(),
                o[4].data_ptr(), None]
        f = L.cq_push_batch_results_noalloc
        assert f(ok._h, k.data_ptr(), k.data_ptr(), cq.NOALLOC_MAX_BATCH + 1, *args) == \
            cq.ERR_INVALID
        assert f(big._h, k.data_ptr(), k.data_ptr(), 10, *args) == cq.ERR_INVALID
        assert f(stat._h, k.data_ptr(), k.data_ptr(), 10, *args) == cq.ERR_INVALID
        assert f(ok._h, None, None, 10, *args) == cq.ERR_INVALID
        assert f(ok._h, k.data_ptr(), k.data_ptr(), 10, *args[:4], None, None) == cq.ERR_INVALID
        # after an allocation-free push the query's own plan is not the last one
        assert f(ok._h, k.data_ptr(), k.data_ptr(), 10, *args) == cq.OK
        torch.cuda.synchronize()
        assert L.cq_results(ok._h, *args) == cq.ERR_INVALID
        assert L.cq_status(ok._h) == cq.ERR_INVALID
        ok.push(k[:10], k[:10])
        assert ok.status() == cq.OK
        ids, sums, counts, avgs = ok.results()
        assert ids.tolist() == [0] and counts.tolist() == [10] and sums.tolist() == [0]
    finally:
        ok.close(), big.close(), stat.close()
