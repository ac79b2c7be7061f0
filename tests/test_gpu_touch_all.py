"""GPU parity when a batch touches every group, at group counts around the
boundaries of the plan paths (16384: plan inside the reorder pass; 16385 ..
32768: a plan launch of its own).  The plan sums per-group fields over the
whole histogram; with every group touched those sums reach their largest
values, which these cases pin bit for bit against the CPU oracle (results,
touched count) in the balanced and static partitions, through the pipelined
entry point, and with keys reduced mod the group count."""
import numpy as np
import pytest

import paper_1309_0634_amd as cq
from gpu_helpers import Pair, assert_same, note, to_dev
from oracle import RingOracle
from test_gpu_pipeline import check_against_oracle
from workloads import probe_batch

pytestmark = pytest.mark.gpu

GROUPS = [16384, 16385, 32767, 32768]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cq.lib()
    torch.cuda.set_device(0)


def every_group_batches(G, seed):
    """A probe batch (each group once), two uniform batches holding every
    group (300,001 and 2^20 tuples: every group appears at least once, the
    ids shuffled in), and the probe again."""
    rng = np.random.default_rng([G, seed])
    out = [probe_batch(G)]
    for n in (300_001, 1 << 20):
        k = rng.integers(0, G, n).astype(np.int32)
        k[rng.permutation(n)[:G]] = rng.permutation(G).astype(np.int32)
        v = rng.integers(-(1 << 31), (1 << 31) - 1, n, endpoint=True).astype(np.int32)
        out.append((k, v))
    out.append(probe_batch(G))
    return out


@pytest.mark.parametrize("G", GROUPS)
@pytest.mark.parametrize("mode,workers", [(cq.PARTITION_BALANCED, 0), (cq.PARTITION_STATIC, 0)],
                         ids=["balanced", "static"])
def test_every_group_touched(G, mode, workers):
    note(f"case: every group touched, G={G}, mode {mode}")
    p = Pair(G, 37, mode, workers)
    for b, (k, v) in enumerate(every_group_batches(G, 1)):
        got = p.step(k, v, f"G={G} mode {mode} batch {b}")
        assert len(got[0]) == G, f"G={G} batch {b}: {len(got[0])} touched, want all {G}"
        plan = p.q.batch_plan()
        assert plan["touched"] == G, f"G={G} batch {b}: plan counts {plan['touched']} touched"
        assert plan["fault"] == 0
    p.close()


@pytest.mark.parametrize("G", GROUPS)
def test_every_group_touched_pipelined(G):
    note(f"case: every group touched, pipelined, G={G}")
    q = cq.Query(G, 37)
    o = RingOracle(G, 37)
    check_against_oracle(q, o, G, every_group_batches(G, 2), f"pipelined G={G}")
    q.close()
    o.close()


@pytest.mark.parametrize("G", GROUPS)
def test_every_group_touched_key_mod(G):
    """Keys over the whole int32 range reduced mod G, every residue present."""
    note(f"case: every group touched, keys mod G={G}")
    rng = np.random.default_rng([G, 3])
    q = cq.Query(G, 37)
    q.set_key_mod(True)
    o = RingOracle(G, 37)
    for b, (k, v) in enumerate(every_group_batches(G, 3)):
        # raw keys with the same residues: k + G * j as uint32, across the range
        j = rng.integers(0, (1 << 32) // G, len(k), dtype=np.int64)
        raw = ((k.astype(np.int64) + G * j) % (1 << 32)).astype(np.uint32).view(np.int32)
        assert np.array_equal(raw.view(np.uint32) % np.uint32(G), k.astype(np.uint32))
        q.push(to_dev(raw), to_dev(v))
        got = q.results()
        want = o.push(k, v)
        assert_same(got, want, f"key mod G={G} batch {b}")
        assert len(got[0]) == G
    q.close()
    o.close()
