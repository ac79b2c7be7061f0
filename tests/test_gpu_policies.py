"""GPU parity under the Section 4 techniques (getFirst .. shiftLocal): the
static workers run every batch with the group-to-worker mapping the host
step derived from the previous batch.  Results must equal the CPU oracle's
bit for bit, and the host step, fed the device histogram, must move exactly
the groups the oracle's techniques move on the same batches."""
import numpy as np
import pytest

import paper_1309_0634_amd as cq
from gpu_helpers import assert_same, note, to_dev
from oracle import OracleError, RingOracle
from oracle import policies as OP
from workloads import host_batch, skew, tiny

pytestmark = pytest.mark.gpu

POLICIES = sorted(OP.NAMES)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cq.lib()
    torch.cuda.set_device(0)


class Tracked:
    """A query under one technique and the oracle's lists for it."""

    def __init__(self, groups, window, policy, workers, threshold, pot=0.5):
        self.q = cq.Query(groups, window)
        self.q.set_policy_params(threshold, pot)
        self.q.set_partition(policy, workers)
        self.policy, self.threshold, self.pot = policy, threshold, pot
        self.groups = groups
        self.lists = OP.initial_lists(workers or 1024, groups)
        self.total = 0

    def expect(self, keys):
        """The oracle's step on this batch: (moves, max tpt, min tpt, total)."""
        counts = np.bincount(keys, minlength=self.groups)
        tpt = OP.tuples_per_thread(self.lists, counts)
        moves = OP.rebalance(self.policy, self.lists, counts.tolist(), self.threshold,
                             self.pot, cq.STATIC_KEYS_MAX, np.asarray(keys).tolist())
        self.total += moves
        return moves, max(tpt), min(tpt), self.total

    def close(self):
        self.q.close()


@pytest.mark.parametrize("policy", POLICIES, ids=lambda p: OP.NAMES[p])
@pytest.mark.parametrize("workers,threshold", [(7, 10), (16, 0), (8, 100), (64, 100)])
def test_tiny_stream_under_technique(policy, workers, threshold):
    """64 groups, W=1000, 4096-tuple batches with a hot key: every batch."""
    note(f"case: tiny stream, {OP.NAMES[policy]}, {workers} workers, threshold {threshold}")
    cfg = tiny()
    o = RingOracle(cfg.groups, cfg.window)
    t = Tracked(cfg.groups, cfg.window, policy, workers, threshold)
    rng = np.random.default_rng([20130909, 91, policy, workers])
    for b in range(24):
        k, v = host_batch(cfg, b)
        k = k.copy()
        k[rng.random(len(k)) < 0.3] = int(rng.integers(0, cfg.groups))  # a hot group
        t.q.push(to_dev(k), to_dev(v))
        assert_same(t.q.results(), o.push(k, v), f"{OP.NAMES[policy]} batch {b}")
        assert t.q.policy_stats() == t.expect(k), f"{OP.NAMES[policy]} batch {b}"
    if workers <= 16:  # (with more, a hot group alone outweighs every gap)
        assert t.total > 0
    t.close()
    o.close()


@pytest.mark.parametrize("s", [0.5, 1.5])
def test_skew_stream_all_techniques(s):
    """10,000 groups, W=1000, 1,048,576-tuple Zipf batches, 1024 workers and
    the paper's threshold of 1000: six batches under every technique."""
    note(f"case: skew stream s={s}, all techniques")
    cfg = skew(s)
    ora = RingOracle(cfg.groups, cfg.window, threads=4)
    ts = [Tracked(cfg.groups, cfg.window, p, 1024, 1000) for p in POLICIES]
    for b in range(6):
        k, v = host_batch(cfg, b)
        dk, dv = to_dev(k), to_dev(v)
        want = ora.push(k, v)
        for t in ts:
            t.q.push(dk, dv)
            assert_same(t.q.results(), want, f"s={s} {OP.NAMES[t.policy]} batch {b}")
            assert t.q.policy_stats() == t.expect(k), f"s={s} {OP.NAMES[t.policy]} batch {b}"
    for t in ts:
        plan = t.q.batch_plan()
        assert plan["fault"] == 0 and plan["status"] == 0
        t.close()
    ora.close()


@pytest.mark.parametrize("policy", [cq.PARTITION_GETFIRST, cq.PARTITION_PROBCHECK,
                                    cq.PARTITION_SHIFT])
def test_pipelined_call_under_technique(policy):
    """cq_push_batches: the host step runs between the batches of one call."""
    import torch
    note(f"case: pipelined call, {OP.NAMES[policy]}")
    cfg = tiny()
    o = RingOracle(cfg.groups, cfg.window)
    t = Tracked(cfg.groups, cfg.window, policy, 9, 20)
    dev = torch.device("cuda", 0)
    hb = [host_batch(cfg, b) for b in range(16)]
    for start in range(0, 16, 8):
        chunk = hb[start:start + 8]
        outs = [(torch.empty(cfg.groups, dtype=torch.int32, device=dev),
                 torch.empty(cfg.groups, dtype=torch.int64, device=dev),
                 torch.empty(cfg.groups, dtype=torch.int32, device=dev),
                 torch.empty(cfg.groups, dtype=torch.float64, device=dev),
                 torch.zeros(1, dtype=torch.int64, device=dev)) for _ in chunk]
        t.q.push_batches_into([(to_dev(k), to_dev(v)) for k, v in chunk], outs)
        torch.cuda.synchronize()
        for i, (k, v) in enumerate(chunk):
            nt = int(outs[i][4].item())
            assert_same(tuple(x[:nt].cpu() for x in outs[i][:4]), o.push(k, v),
                        f"call {start} batch {i}")
            exp = t.expect(k)
        assert t.q.policy_stats() == exp
    t.close()
    o.close()


def test_rejected_batch_moves_nothing():
    note("case: technique with a rejected batch")
    cfg = tiny()
    o = RingOracle(cfg.groups, cfg.window)
    t = Tracked(cfg.groups, cfg.window, cq.PARTITION_CHECKALL, 5, 10)
    for b in range(6):
        k, v = host_batch(cfg, b)
        if b == 3:
            bad = k.copy()
            bad[17] = cfg.groups  # out of range: the whole batch is rejected
            t.q.push(to_dev(bad), to_dev(v))
            with pytest.raises(cq.CQError):
                t.q.results()
            with pytest.raises(OracleError):
                o.push(bad, v)
            assert t.q.policy_stats()[0] == 0
        t.q.push(to_dev(k), to_dev(v))
        assert_same(t.q.results(), o.push(k, v), f"batch {b}")
        assert t.q.policy_stats() == t.expect(k), f"batch {b}"
    t.close()
    o.close()


def test_technique_limits_and_switching():
    note("case: technique limits and mode switches")
    q = cq.Query(40000, 4)
    with pytest.raises(cq.CQError):
        q.set_partition(cq.PARTITION_GETFIRST, 16)  # 2,500 groups per worker
    q.set_partition(cq.PARTITION_GETFIRST, 20)      # 2,000 per worker: taken
    q.close()
    q = cq.Query(4096, 4)
    with pytest.raises(cq.CQError):
        q.set_partition(cq.PARTITION_SHIFT, 1)        # more than 2048 groups per worker
    with pytest.raises(cq.CQError):
        q.set_policy_params(-1, 0.5)
    with pytest.raises(cq.CQError):
        q.set_policy_params(10, 0.0)
    o = RingOracle(4096, 4)
    rng = np.random.default_rng([20130909, 92])
    for b, mode in enumerate([cq.PARTITION_BESTBALANCE, cq.PARTITION_BALANCED,
                              cq.PARTITION_SHIFTLOCAL, cq.PARTITION_STATIC,
                              cq.PARTITION_PROBCHECK]):
        q.set_partition(mode, 3 if mode >= cq.PARTITION_STATIC else 0)
        for i in range(3):
            n = int(rng.integers(1, 30000))
            k = np.minimum(rng.zipf(1.3, n) - 1, 4095).astype(np.int32)
            v = rng.integers(-1000, 1000, n).astype(np.int32)
            q.push(to_dev(k), to_dev(v))
            assert_same(q.results(), o.push(k, v), f"mode {mode} batch {i}")
        stats = q.policy_stats()
        assert (stats == (0, 0, 0, 0)) == (mode < cq.PARTITION_GETFIRST), (mode, stats)
    q.close()
    o.close()
