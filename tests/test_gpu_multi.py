"""GPU parity of queries that share one input stream: keys reduced mod each
query's group count on the device (cq_set_key_mod), and a set of queries
pushed together over several lanes with the online autotuner switching
partitions on live batches (cq_multi_*).  Every query's results must equal
the CPU oracle fed the reduced keys, bit for bit, under every candidate."""
import numpy as np
import pytest

import paper_1309_0634_amd as cq
from gpu_helpers import assert_same, device, note, to_dev
from oracle import RingOracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cq.lib()
    torch.cuda.set_device(0)


def reduced(keys, G):
    return (keys.astype(np.int64) & 0xFFFFFFFF) % G


@pytest.mark.parametrize("G,W", [(1, 3), (7, 5), (1000, 100), (16384, 1000), (20000, 37),
                                 (100000, 10)])
def test_key_mod_matches_reduced_keys(G, W):
    note(f"case: key mod G={G} W={W}")
    import torch
    rng = np.random.default_rng([20130909, 91, G])
    q = cq.Query(G, W)
    q.set_key_mod(True)
    o = RingOracle(G, W)
    for b, n in enumerate([1000, 250000, (1 << 20) + 777, 0, 4096]):
        k = rng.integers(-(1 << 31), (1 << 31) - 1, n, endpoint=True).astype(np.int32)
        v = rng.integers(-1000, 1000, n).astype(np.int32)
        q.push(to_dev(k), to_dev(v))
        assert_same(q.results(), o.push(reduced(k, G).astype(np.int32), v), f"batch {b}")
    # pipelined call (its next histogram rides in the update launch)
    hb = []
    for _ in range(3):
        k = rng.integers(0, 1 << 30, 70000).astype(np.int32)
        hb.append((k, rng.integers(0, 99, 70000).astype(np.int32)))
    outs = [(torch.empty(min(G, 70000), dtype=torch.int32, device=device()),
             torch.empty(min(G, 70000), dtype=torch.int64, device=device()),
             torch.empty(min(G, 70000), dtype=torch.int32, device=device()),
             torch.empty(min(G, 70000), dtype=torch.float64, device=device()),
             torch.empty(1, dtype=torch.int64, device=device())) for _ in hb]
    q.push_batches_into([(to_dev(k), to_dev(v)) for k, v in hb], outs)
    for (k, v), out in zip(hb, outs):
        nt = int(out[4].item())
        assert_same(tuple(t[:nt].cpu() for t in out[:4]),
                    o.push(reduced(k, G).astype(np.int32), v), "pipelined")
    if G <= 16384:  # per-tuple results read the reduced keys the pass staged
        k = rng.integers(-5, 1 << 31, 30000).astype(np.int32)
        v = rng.integers(-9, 9, 30000).astype(np.int32)
        s, c, a = q.push_tuples(to_dev(k), to_dev(v))
        ws, wc, wa = o.push_tuples(reduced(k, G).astype(np.int32), v)
        assert np.array_equal(s.cpu().numpy(), ws) and np.array_equal(c.cpu().numpy(), wc)
        assert np.array_equal(a.cpu().numpy().view(np.int64),
                              np.asarray(wa, np.float64).view(np.int64))
    q.close()
    o.close()


QUERIES = [(100, 10), (257, 1000), (3000, 37), (10000, 1000), (16384, 64), (16385, 500),
           (40000, 200), (65536, 10), (150000, 30), (1000000, 12), (523, 9000), (9000, 1)]


def shared_batches(rng, sizes):
    out = []
    for n in sizes:
        k = rng.zipf(1.3, n) % (1 << 20)
        k = rng.permutation(1 << 20)[k].astype(np.int32)
        out.append((k, rng.integers(0, 1_000_000, n).astype(np.int32)))
    return out


@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_multi_set_with_tuning(lanes):
    note(f"case: multi-query set, {lanes} lanes, tuning")
    rng = np.random.default_rng([20130909, 92, lanes])
    qs = []
    for G, W in QUERIES:
        q = cq.Query(G, W)
        q.set_key_mod(True)
        qs.append(q)
    oras = [RingOracle(G, W, threads=2) for G, W in QUERIES]
    m = cq.Multi(qs, lanes)
    batches = shared_batches(rng, [50000, 300000, 120000, 200000, 90000, 260000, 150000,
                                   (1 << 20) + 4321, 80000, 100000])
    for b, (k, v) in enumerate(batches):
        if b == 1:
            m.tune(2)  # three candidates x 2 batches: batches 1..6
        m.push(to_dev(k), to_dev(v))
        for i, ((G, W), q, o) in enumerate(zip(QUERIES, qs, oras)):
            assert_same(q.results(), o.push(reduced(k, G).astype(np.int32), v),
                        f"batch {b} query {i} (G={G}, W={W})")
    plan = m.plan()
    for (G, _), p in zip(QUERIES, plan):
        assert p["mode"] in (cq.PARTITION_BALANCED, cq.PARTITION_STATIC)
        assert p["mode"] == cq.PARTITION_BALANCED or (G + p["workers"] - 1) // p["workers"] <= 2048
        assert 0 <= p["lane"] < min(lanes, len(QUERIES)) and p["ms"] > 0
    m.close()
    for q, o in zip(qs, oras):
        q.close()
        o.close()


def test_multi_graph_replay():
    """A set replayed as one captured HIP graph per batch size: after every
    replay every query equals the oracle, with eager work and
    synchronisations in between, an eager push on one query of the set
    between replays, a larger batch (new staging, new graphs), an empty
    batch, and a switch back to eager pushes."""
    import torch
    note("case: multi-query graph replay")
    rng = np.random.default_rng([20130909, 93])
    shape = [QUERIES[i] for i in (0, 2, 3, 5, 6, 8, 9, 11)]
    qs = []
    for G, W in shape:
        q = cq.Query(G, W)
        q.set_key_mod(True)
        qs.append(q)
    oras = [RingOracle(G, W, threads=2) for G, W in shape]
    m = cq.Multi(qs, 4)
    other = cq.Query(5000, 50)
    other_o = RingOracle(5000, 50)

    def check(k, v, ctx):
        for i, ((G, W), q, o) in enumerate(zip(shape, qs, oras)):
            assert_same(q.results(), o.push(reduced(k, G).astype(np.int32), v),
                        f"{ctx} query {i} (G={G}, W={W})")

    sizes = [120000, 120000, 60000, 120000, 60000, 0, 60000, (1 << 20) + 999, 120000, 60000]
    batches = shared_batches(rng, [70000, 70000, 70000] + [n for n in sizes] + [40000])
    m.tune(1)
    for b in range(3):
        k, v = batches[b]
        m.push(to_dev(k), to_dev(v))
        check(k, v, f"tuning batch {b}")
    m.set_graph(True)
    for j, (k, v) in enumerate(batches[3:3 + len(sizes)]):
        m.push(to_dev(k), to_dev(v))
        check(k, v, f"replay {j} (n={len(k)})")
        # the program's own eager work between replays
        ok_ = rng.integers(0, 5000, 30000).astype(np.int32)
        ov = rng.integers(0, 100, 30000).astype(np.int32)
        other.push(to_dev(ok_), to_dev(ov))
        assert_same(other.results(), other_o.push(ok_, ov), f"eager work after replay {j}")
        torch.cuda.synchronize()
        if j == 4:  # an eager push on one query of the set, between replays
            G, _ = shape[2]
            ek = rng.integers(0, G, 10000).astype(np.int32)
            ev = rng.integers(0, 100, 10000).astype(np.int32)
            qs[2].push(to_dev(ek), to_dev(ev))
            assert_same(qs[2].results(), oras[2].push(ek, ev), "eager push inside the set")
    m.set_graph(False)
    k, v = batches[-1]
    m.push(to_dev(k), to_dev(v))
    check(k, v, "eager again")
    m.close()
    for q, o in zip(qs, oras):
        q.close()
        o.close()
    other.close()
    other_o.close()
