"""GPU parity at the paper's own setting (Section 5.1): 40,000 groups, W=100,
50,000-tuple batches, on DS1-like (round-robin), DS2-like (Zipf, hot ids
first) and DS3-like (Zipf, permuted) streams.  The Section 4 techniques run
on 1,024 static workers (the paper's grid of 4 blocks of 256 threads) and
on 4,096, the most static workers a partition takes (the paper's grid of 64
blocks has 16,384 threads, about 2.4 groups each; 4,096 workers hold about
ten), threshold 1000, pot 0.5: every batch's results and every host step
against the oracle.  The per-tuple form (a window rescan after every
insertion, once or ten times, Section 5.2) is checked tuple by tuple."""
import numpy as np
import pytest

import paper_1309_0634_amd as cq
from gpu_helpers import assert_same, note, to_dev
from oracle import RingOracle
from oracle import policies as OP
from test_gpu_policies import Tracked
from test_gpu_tuples import check_tuples
from workloads import host_batch, paper_shape

pytestmark = pytest.mark.gpu

POLICIES = sorted(OP.NAMES)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cq.lib()
    torch.cuda.set_device(0)


@pytest.mark.parametrize("dataset", ["DS2", "DS3"])
@pytest.mark.parametrize("workers", [1024, 4096])
def test_paper_shape_techniques(dataset, workers):
    note(f"case: paper shape {dataset}, six techniques on {workers} workers")
    cfg = paper_shape(dataset)
    ora = RingOracle(cfg.groups, cfg.window)
    ts = [Tracked(cfg.groups, cfg.window, p, workers, 1000, 0.5) for p in POLICIES]
    for b in range(5):
        k, v = host_batch(cfg, b)
        dk, dv = to_dev(k), to_dev(v)
        want = ora.push(k, v)
        for t in ts:
            t.q.push(dk, dv)
            assert_same(t.q.results(), want, f"{dataset} {OP.NAMES[t.policy]} batch {b}")
            assert t.q.policy_stats() == t.expect(k), f"{dataset} {OP.NAMES[t.policy]} batch {b}"
    for t in ts:
        plan = t.q.batch_plan()
        assert plan["fault"] == 0 and plan["status"] == 0
        t.close()
    ora.close()


@pytest.mark.parametrize("dataset", ["DS1", "DS2", "DS3"])
def test_paper_shape_static_and_balanced(dataset):
    """No balancing (the static ranges, 1,024 workers) and the device-side
    balanced partition on the same batches."""
    note(f"case: paper shape {dataset}, static and balanced")
    cfg = paper_shape(dataset)
    ora = RingOracle(cfg.groups, cfg.window)
    qs = [cq.Query(cfg.groups, cfg.window, partition=cq.PARTITION_STATIC),
          cq.Query(cfg.groups, cfg.window)]
    for b in range(8):
        k, v = host_batch(cfg, b)
        dk, dv = to_dev(k), to_dev(v)
        want = ora.push(k, v)
        for q in qs:
            q.push(dk, dv)
            assert_same(q.results(), want, f"{dataset} batch {b}")
    for q in qs:
        assert q.batch_plan()["fault"] == 0
        q.close()
    ora.close()


@pytest.mark.parametrize("passes", [0, 1, 10])
@pytest.mark.parametrize("dataset", ["DS1", "DS2", "DS3"])
def test_paper_shape_per_tuple(dataset, passes):
    note(f"case: paper shape {dataset}, per tuple, passes {passes}")
    cfg = paper_shape(dataset)
    q = cq.Query(cfg.groups, cfg.window)
    o = RingOracle(cfg.groups, cfg.window)
    for b in range(4):
        k, v = host_batch(cfg, b)
        check_tuples(q, o, k, v, passes, f"{dataset} batch {b}")
    assert q.batch_plan()["fault"] == 0
    q.close()
    o.close()
