"""GPU parity of cq_push_batches on its several-batch path (up to 16384
groups, balanced partition): up to CHAIN_BATCHES (20) consecutive batches share one
histogram, plan, reorder, survivor and apply launch, and every batch's
results must equal the CPU oracle's bit for bit.  The cases aim at the
path's own structure: windows that span several batches of a call, groups
whose survivors exceed one apply range, apply ranges holding many untouched
groups, rejected batches, calls longer than one set of launches takes, and the
benchmark's own arrays."""
import numpy as np
import pytest

import paper_1309_0634_amd as cq
from gpu_helpers import assert_same, device, note, to_dev
from oracle import RingOracle
from test_gpu_pipeline import check_against_oracle, push_group
from workloads import skew

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cq.lib()
    torch.cuda.set_device(0)


def _rb(rng, G, n, lo=0, hi=10 ** 6, zipf=None):
    if zipf:
        k = (rng.zipf(zipf, n) - 1) % G
    else:
        k = rng.integers(0, G, n)
    return k.astype(np.int32), rng.integers(lo, hi, n).astype(np.int32)


def _no_fault(q):
    plan = q.batch_plan()
    assert plan["fault"] == 0, plan


@pytest.mark.parametrize("W", [1, 2, 3, 7, 100, 1000, 5000])
def test_windows_across_batches(W):
    """Windows that span several batches of a call (small batches, large
    W) and batches longer than the window (small W), sizes ragged."""
    note(f"case: several-batch path, W={W}")
    rng = np.random.default_rng(W)
    G = 300
    q, o = cq.Query(G, W), RingOracle(G, W)
    for call in range(4):
        per = [1, 3, 8, cq.CHAIN_BATCHES][call]
        bs = [_rb(rng, G, int(rng.integers(1, 9000)), -10 ** 6, 10 ** 6,
                  zipf=1.3 if call % 2 else None) for _ in range(per)]
        check_against_oracle(q, o, G, bs, f"W={W} call {call}")
    _no_fault(q)
    q.close(), o.close()


@pytest.mark.parametrize("count", [cq.CHAIN_BATCHES + 1, 2 * cq.CHAIN_BATCHES + 5])
def test_call_longer_than_one_set_of_launches(count):
    """A call of more batches than one set of launches takes: cut into
    near-equal groups (21 = 11 + 10, 45 = 15 + 15 + 15)."""
    note(f"case: several-batch path, {count} batches in one call")
    rng = np.random.default_rng(count)
    G, W = 1000, 64
    q, o = cq.Query(G, W), RingOracle(G, W)
    bs = [_rb(rng, G, int(rng.integers(1, 20000))) for _ in range(count)]
    check_against_oracle(q, o, G, bs, f"{count} batches")
    _no_fault(q)
    q.close(), o.close()


@pytest.mark.parametrize("W,n", [(1000, 60000), (3000, 60000), (200, 200000)])
def test_groups_over_one_apply_range(W, n):
    """Few groups with many tuples: a group's survivors over the call (up to
    twenty windows) plus its old window exceed one apply range and the group
    is summed alone; with W=3000 the windows also reach back across
    batches and into the window before the call."""
    note(f"case: several-batch path, big groups W={W} n={n}")
    rng = np.random.default_rng(W + n)
    G = 50
    q, o = cq.Query(G, W), RingOracle(G, W)
    for call in range(3):
        bs = [_rb(rng, G, n + int(rng.integers(0, 999)), zipf=1.1 if call == 1 else None)
              for _ in range(8 if call == 2 else cq.CHAIN_BATCHES)]
        check_against_oracle(q, o, G, bs, f"W={W} call {call}")
    _no_fault(q)
    q.close(), o.close()


def test_sparse_groups_many_untouched_per_range():
    """16384 groups of which only every 37th is ever touched: apply ranges
    hold many more groups than survivors."""
    note("case: several-batch path, sparse keys over 16384 groups")
    rng = np.random.default_rng(37)
    G, W = 16384, 5
    q, o = cq.Query(G, W), RingOracle(G, W)
    live = np.arange(0, G, 37)
    for call in range(3):
        bs = []
        for _ in range(6):
            n = int(rng.integers(1000, 50000))
            bs.append((live[rng.integers(0, len(live), n)].astype(np.int32),
                       rng.integers(0, 10 ** 6, n).astype(np.int32)))
        check_against_oracle(q, o, G, bs, f"sparse call {call}")
    _no_fault(q)
    q.close(), o.close()


def test_group_touched_only_by_a_rejected_batch():
    """A rejected batch's counts must not leak into the next call, also for
    a group that no accepted batch touches."""
    note("case: several-batch path, counts of a rejected batch")
    rng = np.random.default_rng(3)
    G, W = 500, 20
    q, o = cq.Query(G, W), RingOracle(G, W)
    good = [_rb(rng, G - 1, 3000) for _ in range(3)]  # group G-1 untouched
    bad_k = np.full(4000, G - 1, np.int32)
    bad_k[100] = G + 5  # out of range
    bad = (bad_k, rng.integers(0, 10 ** 6, 4000).astype(np.int32))
    check_against_oracle(q, o, G, [good[0], bad, good[1]], "with rejection")
    check_against_oracle(q, o, G, [good[2], _rb(rng, G, 5000)], "after rejection")
    # everything rejected, then a normal call
    check_against_oracle(q, o, G, [bad, bad], "all rejected")
    check_against_oracle(q, o, G, [_rb(rng, G, 7000) for _ in range(5)], "after all rejected")
    _no_fault(q)
    q.close(), o.close()


def test_key_mod_and_results_after_the_call():
    note("case: several-batch path with key reduction; cq_results after it")
    rng = np.random.default_rng(77)
    G, W = 1234, 50
    q, o = cq.Query(G, W), RingOracle(G, W)
    q.set_key_mod(True)
    for call in range(3):
        raw = [(rng.integers(-2 ** 31, 2 ** 31 - 1, n, dtype=np.int64).astype(np.int32),
                rng.integers(0, 10 ** 6, n).astype(np.int32))
               for n in rng.integers(1, 30000, 5)]
        got = push_group(q, G, raw)
        for i, ((k, v), g) in enumerate(zip(raw, got)):
            want = o.push((k.view(np.uint32) % G).astype(np.int32), v)
            assert_same(g, want, f"key-mod call {call} batch {i}")
        # cq_results emits the call's last batch again
        assert_same(q.results(), want, f"results after call {call}")
        assert q.status() == cq.OK
    _no_fault(q)
    q.close(), o.close()


@pytest.mark.parametrize("s", [0.0, 0.5, 1.0, 1.5, 2.0])
def test_bench_arrays_whole_chains_per_call(s):
    """The benchmark's timed configuration: its 200 device-drawn batches of
    the 10,000-group, W=1000, 2^20-tuple Zipf stream in the order it cycles
    them (200, then the first 10 again), CHAIN_BATCHES per call, every
    batch's results against the oracle's."""
    import torch
    from workloads import DeviceStream
    note(f"case: bench arrays s={s}, {cq.CHAIN_BATCHES} batches per call")
    cfg = skew(s)
    ds = DeviceStream(cfg, device())
    q = cq.Query(cfg.groups, cfg.window)
    o = RingOracle(cfg.groups, cfg.window, threads=4)
    dev = device()
    seqn = list(range(cfg.batches)) + list(range(10))
    pc = cq.CHAIN_BATCHES
    for c0 in range(0, len(seqn), pc):
        idx = seqn[c0:c0 + pc]
        dbs = [ds.batch(b) for b in idx]
        outs = [(torch.empty(cfg.groups, dtype=torch.int32, device=dev),
                 torch.empty(cfg.groups, dtype=torch.int64, device=dev),
                 torch.empty(cfg.groups, dtype=torch.int32, device=dev),
                 torch.empty(cfg.groups, dtype=torch.float64, device=dev),
                 torch.empty(1, dtype=torch.int64, device=dev)) for _ in idx]
        q.push_batches_into(dbs, outs)
        torch.cuda.synchronize()
        for j, ((dk, dv), out) in enumerate(zip(dbs, outs)):
            want = o.push(dk.cpu().numpy(), dv.cpu().numpy())
            nt = int(out[4].item())
            assert_same(tuple(t[:nt].cpu() for t in out[:4]), want,
                        f"s={s} push {c0 + j} (batch {idx[j]})")
    _no_fault(q)
    q.close(), o.close()


@pytest.mark.parametrize("G,W", [(1, 1), (1, 3), (2, 1), (3, 4096)])
def test_degenerate_shapes(G, W):
    """One to three groups (every key the same few), windows of 1 to 4096,
    batches of 0, 1 and 2^20 tuples inside one call."""
    note(f"case: several-batch path, G={G} W={W}")
    rng = np.random.default_rng([G, W])
    q, o = cq.Query(G, W), RingOracle(G, W)
    sizes = [0, 1, 1 << 20, 5, 0, 70000, 1, 3, 2, 0, 1 << 20, 1, 9000, 0, 4, 1, 7, 0, 1, 2]
    bs = [(rng.integers(0, G, n).astype(np.int32), rng.integers(-10 ** 6, 10 ** 6, n).astype(np.int32))
          for n in sizes]
    check_against_oracle(q, o, G, bs, f"G={G} W={W}")
    check_against_oracle(q, o, G, bs[:3], f"G={G} W={W} again")
    _no_fault(q)
    q.close(), o.close()


def test_every_group_touched_at_the_group_limit():
    """16,384 groups, each touched in every batch (a probe of all groups
    plus random keys), W=2 and W=700, so every group's window turns over."""
    from workloads import probe_batch
    for W in (2, 700):
        note(f"case: several-batch path, all 16384 groups touched, W={W}")
        rng = np.random.default_rng(W)
        G = 16384
        q, o = cq.Query(G, W), RingOracle(G, W)
        pk, pv = probe_batch(G)
        bs = []
        for i in range(cq.CHAIN_BATCHES):
            k = np.concatenate([pk, rng.integers(0, G, 40000).astype(np.int32)])
            v = np.concatenate([pv, rng.integers(0, 10 ** 6, 40000).astype(np.int32)])
            bs.append((k, v))
        check_against_oracle(q, o, G, bs, f"all touched W={W}")
        _no_fault(q)
        q.close(), o.close()
