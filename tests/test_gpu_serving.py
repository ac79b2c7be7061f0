"""GPU tests of the serving loop (cq_server_*): resident queries admitted by
device footprint, batches submitted while others run on the device.  Every
request's results must be bit-identical to the CPU oracle's and to the same
query run alone (cq_push_batch_results on a query of its own)."""
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


QUERIES = [(50, 5), (300, 100), (2000, 1000), (20000, 37), (100000, 10), (1000, 1),
           (16384, 1000), (40000, 300)]


def make_batches(rng, G, count, big=False):
    out = []
    for b in range(count):
        n = int(rng.choice([0, 1, 37, 4096, 50000, 150000]))
        if big and b == 2:
            n = (1 << 20) + 12345  # more than one sub-batch
        k = np.minimum(rng.zipf(1.4, n) - 1, G - 1).astype(np.int32)
        k = rng.permutation(G).astype(np.int32)[k] if n else k
        v = rng.integers(-(1 << 31), (1 << 31) - 1, n, endpoint=True).astype(np.int32)
        out.append((k, v))
    return out


def outputs(G, n):
    import torch
    cap = max(1, min(G, n))
    dev = device()
    return (torch.empty(cap, dtype=torch.int32, device=dev),
            torch.empty(cap, dtype=torch.int64, device=dev),
            torch.empty(cap, dtype=torch.int32, device=dev),
            torch.empty(cap, dtype=torch.float64, device=dev),
            torch.full((1,), -99, dtype=torch.int64, device=dev))


def got_of(o):
    nt = int(o[4].item())
    return nt if nt < 0 else tuple(t[:nt].cpu() for t in o[:4])


@pytest.mark.parametrize("lanes,slots", [(4, 2), (16, 1), (1, 64)])
def test_results_same_alone_and_in_the_mix(lanes, slots):
    note(f"case: serving mix, {lanes} lanes x {slots} slots")
    rng = np.random.default_rng([20130909, 71, lanes])
    srv = cq.Server(0, lanes, slots)
    qids = [srv.add_query(G, W) for G, W in QUERIES]
    batches = [make_batches(rng, G, 6, big=(i == 3)) for i, (G, _) in enumerate(QUERIES)]
    dev_b = [[(to_dev(k), to_dev(v)) for k, v in bs] for bs in batches]
    outs = [[outputs(G, len(k)) for k, _ in bs] for (G, _), bs in zip(QUERIES, batches)]
    # interleave submissions across queries, each query in its own order
    order = [i for i, bs in enumerate(batches) for _ in bs]
    rng.shuffle(order)
    nxt = [0] * len(QUERIES)
    tickets = []
    for i in order:
        b = nxt[i]
        nxt[i] += 1
        k, v = dev_b[i][b]
        ids, sums, counts, avgs, nt = outs[i][b]
        tickets.append(srv.submit(qids[i], k, v, ids, sums, counts, avgs, nt))
    for t in tickets[::2]:
        srv.wait(t)
    srv.wait()
    st = srv.stats()
    assert st["requests"] == len(order)
    assert st["tuples"] == sum(len(k) for bs in batches for k, _ in bs)
    assert 0 < st["p50_us"] <= st["p99_us"] <= st["max_us"]
    for i, (G, W) in enumerate(QUERIES):
        alone = cq.Query(G, W)
        ora = RingOracle(G, W)
        for b, (k, v) in enumerate(batches[i]):
            want = ora.push(k, v)
            got = got_of(outs[i][b])
            assert not isinstance(got, int), f"query {i} batch {b}: status {got}"
            assert_same(got, want, f"served query {i} ({G},{W}) batch {b}")
            o = outputs(G, len(k))
            alone.push_results_into(dev_b[i][b][0], dev_b[i][b][1], *o)
            assert_same(got_of(o), want, f"alone query {i} batch {b}")
        alone.close()
        ora.close()
    srv.close()


def test_admission_by_footprint():
    note("case: serving admission")
    fa, fb, fc = (cq.query_footprint(*q) for q in [(10000, 1000), (5000, 100), (12000, 800)])
    assert 4096 < fc <= fa
    srv = cq.Server(fa + fb + 4096, 2, 2)
    a = srv.add_query(10000, 1000)
    b = srv.add_query(5000, 100)
    assert srv.stats()["bytes_held"] == fa + fb
    with pytest.raises(cq.CQError) as e:
        srv.add_query(12000, 800)
    assert e.value.code == cq.ERR_OOM
    srv.remove_query(a)
    c = srv.add_query(12000, 800)  # fits in the freed room
    assert srv.stats()["bytes_held"] == fb + fc
    k = to_dev(np.arange(100, dtype=np.int32) % 5000)
    v = to_dev(np.ones(100, dtype=np.int32))
    with pytest.raises(cq.CQError):
        srv.submit(a, k, v)  # removed
    t = srv.submit(c, k, v)
    srv.wait(t)
    with pytest.raises(cq.CQError):
        srv.wait(t)  # a ticket is waited for once
    with pytest.raises(cq.CQError):
        srv.wait(10 ** 9)
    srv.remove_query(b)
    srv.remove_query(c)
    assert srv.stats()["bytes_held"] == 0
    srv.close()


def test_rejected_batch_in_the_mix():
    note("case: serving rejected batch")
    rng = np.random.default_rng([20130909, 72])
    srv = cq.Server(0, 3, 2)
    G, W = 500, 20
    qa, qb = srv.add_query(G, W), srv.add_query(G, W)
    oa, ob = RingOracle(G, W), RingOracle(G, W)
    reqs = []
    for b in range(5):
        for q, o in ((qa, oa), (qb, ob)):
            k = rng.integers(0, G, 3000).astype(np.int32)
            v = rng.integers(-50, 50, 3000).astype(np.int32)
            bad = b == 2 and q == qa
            if bad:
                k[1500] = G
            out = outputs(G, 3000)
            srv.submit(q, to_dev(k), to_dev(v), *out)
            reqs.append((o, k, v, out, bad))
    srv.wait()
    for o, k, v, out, bad in reqs:
        got = got_of(out)
        if bad:
            assert got == cq.ERR_KEY_RANGE
        else:
            assert_same(got, o.push(k, v), "mixed request")
    srv.close()


def test_concurrent_submitters_and_churn():
    """Four caller threads submit to their own queries at once while a fifth
    adds and removes queries; every request equals the oracle."""
    note("case: serving, concurrent submitters")
    import threading
    srv = cq.Server(0, 4, 2)
    shapes = [(500, 20), (7000, 300), (30000, 64), (120000, 5)]
    qids = [srv.add_query(G, W) for G, W in shapes]
    rng = np.random.default_rng([20130909, 73])
    work = [make_batches(np.random.default_rng([20130909, 74, i]), G, 10)
            for i, (G, _) in enumerate(shapes)]
    dev_w = [[(to_dev(k), to_dev(v)) for k, v in bs] for bs in work]
    outs = [[outputs(G, len(k)) for k, _ in bs] for (G, _), bs in zip(shapes, work)]
    errors = []

    def submitter(i):
        try:
            for b, (k, v) in enumerate(dev_w[i]):
                srv.submit(qids[i], k, v, *outs[i][b])
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(e)

    def churn():
        try:
            for j in range(6):
                q = srv.add_query(int(rng.integers(100, 5000)), int(rng.integers(1, 50)))
                k = to_dev(np.zeros(10, np.int32))
                srv.wait(srv.submit(q, k, k))
                srv.remove_query(q)
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(e)

    threads = [threading.Thread(target=submitter, args=(i,)) for i in range(len(shapes))]
    threads.append(threading.Thread(target=churn))
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    srv.wait()
    for i, (G, W) in enumerate(shapes):
        o = RingOracle(G, W)
        for b, (k, v) in enumerate(work[i]):
            got = got_of(outs[i][b])
            assert not isinstance(got, int), f"query {i} batch {b}: status {got}"
            assert_same(got, o.push(k, v), f"concurrent query {i} batch {b}")
        o.close()
    srv.close()
