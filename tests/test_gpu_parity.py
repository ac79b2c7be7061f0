"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle,
bit for bit (ids, int64 sums, counts, and the binary64 AVG bit patterns).

Integer work and a single correctly rounded division: the bar is exact
equality, tolerance 0."""
import numpy as np
import pytest

import paper_1309_0634_amd as cq
from gpu_helpers import Pair, assert_same, device, note, to_dev
from oracle import RingOracle
from workloads import (DeviceStream, StreamConfig, drifting, host_batch, probe_batch, skew,
                       tiny)

pytestmark = pytest.mark.gpu

MODES = [(cq.PARTITION_BALANCED, 0), (cq.PARTITION_STATIC, 0), (cq.PARTITION_STATIC, 7)]
MODE_IDS = ["balanced", "static1024", "static7"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cq.lib()
    torch.cuda.set_device(0)


def test_smoke_tiny_eight_batches():
    note("case: tiny stream, 8 batches, balanced")
    p = Pair(64, 1000)
    cfg = tiny()
    for b in range(8):
        k, v = host_batch(cfg, b)
        p.step(k, v, f"tiny batch {b}")
    p.close()


@pytest.mark.parametrize("mode,workers", MODES, ids=MODE_IDS)
def test_tiny_config_all_batches(mode, workers):
    """64 groups, W=1000, 100 batches of 4096 uniform keys: every batch."""
    note(f"case: tiny stream, 100 batches, mode {mode} workers {workers}")
    cfg = tiny()
    p = Pair(cfg.groups, cfg.window, mode, workers)
    for b in range(cfg.batches):
        k, v = host_batch(cfg, b)
        p.step(k, v, f"tiny batch {b}")
    p.close()


@pytest.mark.parametrize("W", [1, 2, 3, 7])
def test_tiny_windows_wrap_many_times(W):
    note(f"case: small windows W={W}")
    rng = np.random.default_rng(W)
    for mode, workers in MODES:
        p = Pair(37, W, mode, workers)
        for b in range(12):
            n = int(rng.integers(0, 3000))
            k = rng.integers(0, 37, n).astype(np.int32)
            v = rng.integers(-(1 << 31), (1 << 31) - 1, n, endpoint=True).astype(np.int32)
            p.step(k, v, f"W={W} mode {mode} batch {b}")
        p.close()


def test_single_group_heavy_batches():
    """G=1: every tuple on one key; batches far longer than the window."""
    note("case: one group, heavy batches")
    rng = np.random.default_rng(5)
    for W in (1, 100, 1000, 1023, 1024, 1025, 5000):
        for mode, workers in MODES[:2]:
            p = Pair(1, W, mode, workers)
            for n in (0, 1, 5, 511, 512, 513, 1023, 1024, 2047, 2048, 2049, 4096 * 3 + 17,
                      100_000):
                k = np.zeros(n, np.int32)
                v = rng.integers(-1000, 1000, n).astype(np.int32)
                p.step(k, v, f"G=1 W={W} n={n} mode {mode}")
            p.close()


def test_heavy_groups_with_large_window():
    """Heavy groups whose surviving tail spans many arrival tiles and many
    chunks (W = 10000, k_g up to 60000)."""
    note("case: large window heavy groups")
    rng = np.random.default_rng(6)
    G, W = 50, 10_000
    for mode, workers in MODES[:2]:
        p = Pair(G, W, mode, workers)
        for b in range(6):
            n = 200_000
            # a few very hot keys plus background
            k = np.where(rng.random(n) < 0.6, rng.integers(0, 3, n), rng.integers(0, G, n))
            k = k.astype(np.int32)
            v = rng.integers(0, 1_000_000, n).astype(np.int32)
            p.step(k, v, f"W=10000 batch {b} mode {mode}")
        p.close()


@pytest.mark.parametrize("G", [1000, 32768, 32769, 100_000, 2_621_440, 2_621_441, 3_000_000])
def test_histogram_paths(G):
    """Direct-indexed LDS counters (G <= 32768) with the plan inside the
    reorder pass or in a launch of its own, and the LDS hash with the
    multi-block plan (larger G): block sums, then the per-group writes with
    every block scanning the sums itself (up to 1024 blocks of 2560 groups,
    G <= 2,621,440), or with a scan launch between them (beyond)."""
    note(f"case: histogram path G={G}")
    rng = np.random.default_rng(G)
    p = Pair(G, 64)
    for b in range(5):
        n = int(rng.integers(1, 300_000))
        k = rng.integers(0, G, n).astype(np.int32)
        if b % 2:
            k[: n // 3] = rng.integers(0, 4, n // 3)
        v = rng.integers(-5, 5, n).astype(np.int32)
        p.step(k, v, f"G={G} batch {b}")
    p.close()


def test_unaligned_and_ragged_inputs():
    """Inputs that are not 16-byte aligned and sizes that are not multiples
    of anything: the scalar load path."""
    note("case: unaligned inputs")
    import torch
    rng = np.random.default_rng(9)
    p = Pair(333, 17)
    for b, n in enumerate([1, 2, 3, 4, 5, 2047, 2049, 6151, 70001]):
        k = rng.integers(0, 333, n + 1).astype(np.int32)
        v = rng.integers(0, 99, n + 1).astype(np.int32)
        dk, dv = to_dev(k)[1:], to_dev(v)[1:]
        p.step(k[1:], v[1:], f"unaligned n={n}", dkeys=dk, dvalues=dv)
    p.close()


@pytest.mark.parametrize("G", [100, 20_000, 100_000, 3_000_000],
                         ids=["in-pass-plan", "plan-launch", "two-launch-plan",
                              "three-launch-plan"])
def test_bad_key_rejects_batch_and_keeps_state(G):
    """A bad key rejects its whole batch and leaves every window as it was,
    on each of the four plan paths."""
    note(f"case: bad key G={G}")
    import torch
    rng = np.random.default_rng(11)
    W = 5
    p = Pair(G, W)
    k = rng.integers(0, G, 5000).astype(np.int32)
    v = rng.integers(0, 100, 5000).astype(np.int32)
    p.step(k, v, "before")
    for bad in (G, -1, 1 << 30):
        kb = rng.integers(0, G, 3000).astype(np.int32)
        kb[1234] = bad
        vb = rng.integers(0, 100, 3000).astype(np.int32)
        p.q.push(to_dev(kb), to_dev(vb))
        with pytest.raises(cq.CQError) as e:
            p.q.results()
        assert e.value.code == cq.ERR_KEY_RANGE
        assert p.q.status() == cq.ERR_KEY_RANGE
        nt = torch.empty(1, dtype=torch.int64, device=device())
        ids = torch.full((10,), -7, dtype=torch.int32, device=device())
        p.q.results_into(ids, None, None, None, nt)
        assert int(nt.item()) == cq.ERR_KEY_RANGE
        assert (ids.cpu() == -7).all()
    for b in range(4):
        k = rng.integers(0, G, 4000).astype(np.int32)
        v = rng.integers(0, 100, 4000).astype(np.int32)
        p.step(k, v, f"after reject {b}")
    assert p.q.status() == cq.OK
    p.close()


def test_empty_batch_and_results_before_push():
    note("case: empty batch")
    import torch
    p = Pair(10, 3)
    nt = torch.full((1,), 99, dtype=torch.int64, device=device())
    p.q.results_into(None, None, None, None, nt)
    assert int(nt.item()) == 0
    e = np.zeros(0, np.int32)
    p.step(e, e, "empty first")
    k = np.array([1, 2, 1, 9], np.int32)
    v = np.array([4, 5, 6, 7], np.int32)
    p.step(k, v, "after empty")
    p.step(e, e, "empty again")
    p.step(k, v, "again")
    p.close()


def test_probe_exposes_identical_windows():
    """After the same stream, probing every group W times returns the same
    windows on both sides (the state, not just the last results)."""
    note("case: probe")
    cfg = tiny()
    p = Pair(cfg.groups, 50)
    for b in range(10):
        k, v = host_batch(cfg, b)
        p.step(k, v, f"stream {b}")
    pk, pv = probe_batch(cfg.groups)
    for j in range(50):
        p.step(pk, pv, f"probe {j}")
    p.close()


@pytest.mark.parametrize("s", [0.0, 0.5, 1.0, 1.5, 2.0])
def test_skew_config_prefix_all_modes(s):
    """10,000 groups, W=1000, 1,048,576-tuple Zipf batches: the first 12
    batches, balanced and static partitions against one oracle run."""
    note(f"case: skew stream s={s}, 12 batches, all modes")
    cfg = skew(s)
    qs = [cq.Query(cfg.groups, cfg.window, partition=m, workers=w) for m, w in MODES]
    ora = RingOracle(cfg.groups, cfg.window, threads=4)
    for b in range(12):
        k, v = host_batch(cfg, b)
        dk, dv = to_dev(k), to_dev(v)
        want = ora.push(k, v)
        for (m, w), q in zip(MODES, qs):
            q.push(dk, dv)
            assert_same(q.results(), want, f"s={s} batch {b} mode {m}/{w}")
    for q in qs:
        plan = q.batch_plan()
        assert plan["fault"] == 0 and plan["status"] == 0
        q.close()


@pytest.mark.parametrize("s", [0.0, 0.5, 1.0, 1.5, 2.0])
def test_skew_config_full_run_balanced(s):
    """The whole timed configuration: all 200 batches of the 10,000-group,
    W=1000, 1,048,576-tuple Zipf stream under the balanced partition, every
    batch's results against the oracle's."""
    note(f"case: skew stream s={s}, all 200 batches, balanced")
    cfg = skew(s)
    p = Pair(cfg.groups, cfg.window, oracle_threads=4)
    for b in range(cfg.batches):
        k, v = host_batch(cfg, b)
        p.step(k, v, f"s={s} batch {b}")
    plan = p.q.batch_plan()
    assert plan["fault"] == 0 and plan["status"] == 0
    p.close()


@pytest.mark.parametrize("s", [0.0, 0.5, 1.0, 1.5, 2.0])
def test_skew_bench_arrays_full_run_balanced(s):
    """The arrays the benchmark times: its 200 device-drawn batches of the
    10,000-group, W=1000, 1,048,576-tuple Zipf stream (DeviceStream), in the
    order the benchmark cycles them (all 200, then the first 10 again), each
    batch copied to the host for the oracle."""
    note(f"case: bench arrays s={s}, 210 pushes, balanced")
    from workloads import DeviceStream
    cfg = skew(s)
    ds = DeviceStream(cfg, device())
    p = Pair(cfg.groups, cfg.window, oracle_threads=4)
    for i in range(cfg.batches + 10):
        dk, dv = ds.batch(i % cfg.batches)
        k, v = dk.cpu().numpy(), dv.cpu().numpy()
        p.step(k, v, f"bench arrays s={s} push {i}", dkeys=dk, dvalues=dv)
    plan = p.q.batch_plan()
    assert plan["fault"] == 0 and plan["status"] == 0
    p.close()


def test_skew_config_full_run_static():
    """All 200 batches of the s=1.5 skew stream under the static partition
    (the baseline the benchmark reports beside the balanced one)."""
    note("case: skew stream s=1.5, all 200 batches, static")
    cfg = skew(1.5)
    p = Pair(cfg.groups, cfg.window, cq.PARTITION_STATIC, 0, oracle_threads=4)
    for b in range(cfg.batches):
        k, v = host_batch(cfg, b)
        p.step(k, v, f"static s=1.5 batch {b}")
    plan = p.q.batch_plan()
    assert plan["fault"] == 0 and plan["status"] == 0
    p.close()


def test_skew_sorted_ids_worst_case_for_static():
    """DS2-like order (hot keys are the smallest ids): the static worker that
    owns the first range gets nearly all the load; results stay identical."""
    note("case: skew s=1.5 unpermuted")
    cfg = skew(1.5, permuted=False)
    p = Pair(cfg.groups, cfg.window, cq.PARTITION_STATIC, 0, oracle_threads=4)
    q2 = cq.Query(cfg.groups, cfg.window)
    for b in range(8):
        k, v = host_batch(cfg, b)
        dk, dv = to_dev(k), to_dev(v)
        got = p.step(k, v, f"sorted batch {b}", dkeys=dk, dvalues=dv)
        q2.push(dk, dv)
        got2 = q2.results()
        for a, c in zip(got, got2):
            assert np.array_equal(a.numpy(), c.numpy())
    p.close()
    q2.close()


def _plan_constant(name):
    """A balancer constant of the HIP path (its internal header)."""
    import os
    import re
    src = open(os.path.join(os.path.dirname(cq.__file__), "csrc", "cq_internal.h")).read()
    return int(re.search(r"constexpr int %s = (\d+);" % name, src).group(1))


def test_partition_plan_matches_histogram():
    """The balancer's plan equals what numpy derives from the histogram:
    groups with >= HEAVY_MIN tuples are heavy buckets, the rest are packed
    into buckets of LIGHT_BUDGET tuples."""
    note("case: plan totals")
    hmin, budget = _plan_constant("HEAVY_MIN"), _plan_constant("LIGHT_BUDGET")
    cfg = skew(1.5)
    q = cq.Query(cfg.groups, cfg.window)
    for b in range(3):
        k, v = host_batch(cfg, b)
        q.push(to_dev(k), to_dev(v))
        plan = q.batch_plan()
        kk = np.bincount(k, minlength=cfg.groups)
        light = (kk > 0) & (kk < hmin)
        heavy = kk >= hmin
        nl = (int(kk[light].sum()) + budget - 1) // budget
        assert plan["touched"] == int((kk > 0).sum()) == plan["sub_touched"]
        assert plan["heavy_groups"] == int(heavy.sum())
        assert plan["light_tuples"] == int(kk[light].sum())
        assert plan["light_buckets"] == nl
        assert plan["buckets"] == nl + int(heavy.sum())
        assert plan["tiles"] == (len(k) + 4095) // 4096 and plan["fault"] == 0
    q.set_partition(cq.PARTITION_STATIC, 100)
    k, v = host_batch(cfg, 3)
    q.push(to_dev(k), to_dev(v))
    plan = q.batch_plan()
    assert plan["buckets"] == 100 and plan["heavy_groups"] == 0
    assert plan["light_tuples"] == len(k)
    q.close()


def test_fused_push_results_matches_split_calls():
    """cq_push_batch_results gives the same results as cq_push_batch then
    cq_results, also across sub-batch boundaries."""
    note("case: fused push+results")
    import torch
    rng = np.random.default_rng(21)
    G, W = 3000, 64
    a = Pair(G, W)
    q = cq.Query(G, W)
    dev = device()
    for b, n in enumerate([100, 70_000, (1 << 20) + 5, 3 * (1 << 20) - 7, 0, 12]):
        k = rng.integers(0, G, n).astype(np.int32)
        k[: n // 2] = rng.integers(0, 5, n // 2)
        v = rng.integers(-50, 50, n).astype(np.int32)
        dk, dv = to_dev(k), to_dev(v)
        want = a.step(k, v, f"split n={n}", dkeys=dk, dvalues=dv)
        cap = max(1, min(G, n))
        ids = torch.empty(cap, dtype=torch.int32, device=dev)
        sums = torch.empty(cap, dtype=torch.int64, device=dev)
        cnts = torch.empty(cap, dtype=torch.int32, device=dev)
        avgs = torch.empty(cap, dtype=torch.float64, device=dev)
        nt = torch.empty(1, dtype=torch.int64, device=dev)
        q.push_results_into(dk, dv, ids, sums, cnts, avgs, nt)
        m = int(nt.item())
        got = (ids[:m].cpu(), sums[:m].cpu(), cnts[:m].cpu(), avgs[:m].cpu())
        for x, y in zip(got, want):
            assert np.array_equal(x.numpy().view(np.int64) if x.dtype == torch.float64 else x.numpy(),
                                  y.numpy().view(np.int64) if y.dtype == torch.float64 else y.numpy())
    a.close()
    q.close()


@pytest.mark.parametrize("mode,G,s", [(cq.PARTITION_STATIC, 10_000, 0.0),
                                       (cq.PARTITION_STATIC, 16_384, 1.5),
                                       (cq.PARTITION_STATIC, 40_000, 1.0),
                                       (cq.PARTITION_BALANCED, 16_384, 0.0),
                                       (cq.PARTITION_BALANCED, 40_000, 0.5)],
                         ids=["static4096-g10000-s0", "static4096-g16384-s1.5",
                              "static4096-g40000-s1", "balanced-g16384-s0",
                              "balanced-g40000-s0.5"])
def test_most_buckets_per_pass(mode, G, s):
    """The most buckets a reorder pass sees: a static partition of 4096
    workers (bucket ids up to 4095, every entry of the multisplit's per-wave
    leader table) and uniform keys under the balanced partition (about 2048
    light buckets), on the in-block plan (G <= 16384) and the separate one;
    batches ragged across tiles and sub-batches."""
    note(f"case: most buckets mode {mode} G={G} s={s}")
    cfg = StreamConfig(f"most_buckets_g{G}_s{s:g}", 9, G, 300, 1 << 20, 3,
                       "zipf" if s > 0 else "uniform", zipf_s=s, s_index=int(s * 10))
    p = Pair(G, cfg.window, mode, 4096 if mode == cq.PARTITION_STATIC else 0, oracle_threads=4)
    for b, n in enumerate([(1 << 20) + 13, 300_001, 4096 * 5 + 1]):
        k, v = host_batch(cfg, b, n)
        p.step(k, v, f"most buckets batch {b} (n={n})")
    p.close()


def test_static_partition_limits():
    note("case: static limits")
    q = cq.Query(1 << 20, 4)
    with pytest.raises(cq.CQError):
        q.set_partition(cq.PARTITION_STATIC, 100)   # more than 2048 groups per worker
    with pytest.raises(cq.CQError):
        q.set_partition(cq.PARTITION_STATIC, 5000)  # more workers than buckets
    q.set_partition(cq.PARTITION_STATIC, 1024)
    q.close()


def test_determinism_same_input_twice():
    note("case: determinism")
    cfg = skew(1.0)
    a = cq.Query(cfg.groups, cfg.window)
    b_ = cq.Query(cfg.groups, cfg.window)
    for b in range(6):
        k, v = host_batch(cfg, b)
        dk, dv = to_dev(k), to_dev(v)
        a.push(dk, dv)
        ra = a.results()
        b_.push(dk, dv)
        rb = b_.results()
        for x, y in zip(ra, rb):
            assert np.array_equal(x.numpy(), y.numpy())
    a.close()
    b_.close()


def test_independent_queries_interleaved():
    note("case: two queries")
    rng = np.random.default_rng(3)
    p1 = Pair(500, 9)
    p2 = Pair(70, 400)
    for b in range(6):
        k1 = rng.integers(0, 500, 20_000).astype(np.int32)
        k2 = rng.integers(0, 70, 30_000).astype(np.int32)
        v1 = rng.integers(0, 100, 20_000).astype(np.int32)
        v2 = rng.integers(0, 100, 30_000).astype(np.int32)
        p1.step(k1, v1, f"q1 {b}")
        p2.step(k2, v2, f"q2 {b}")
    p1.close()
    p2.close()


def test_drifting_config_full_size_across_redraws():
    """2^20 groups, W=100, 16,777,216-tuple batches (Zipf s=1.2, clipped
    normal values) with the hot-key permutation redrawn every 3 batches, so
    the redraws at batches 3 and 6 are crossed at full size."""
    note("case: drifting stream, full-size batches, 8 batches")
    import torch
    base = drifting()
    cfg = StreamConfig(base.name + "_epoch3", base.config_id, base.groups, base.window,
                       base.batch, 8, base.key_dist, zipf_s=base.zipf_s, permuted=True,
                       perm_epoch=3, value_dist=base.value_dist, s_index=7)
    ds = DeviceStream(cfg, device())
    p = Pair(cfg.groups, cfg.window, oracle_threads=8)
    for b in range(cfg.batches):
        dk, dv = ds.batch(b)
        k, v = dk.cpu().numpy(), dv.cpu().numpy()
        p.step(k, v, f"drift batch {b}", dkeys=dk, dvalues=dv)
        note(f"  drift batch {b} ok")
    plan = p.q.batch_plan()
    assert plan["fault"] == 0
    p.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("G,n", [(16384, 5000), (16384, 300_000), (10, 1 << 20), (3, 20_000),
                                 (12_345, 4096 * 7 + 5)],
                         ids=["maxG-2tiles", "maxG-74tiles", "G10-256tiles", "G3", "ragged"])
def test_in_pass_plan_ownership(G, n):
    """The plan inside the reorder pass: each workgroup owns a contiguous
    range of groups (several passes when a small grid owns many, none when
    the grid outnumbers the groups)."""
    note(f"case: in-pass plan ownership G={G} n={n}")
    rng = np.random.default_rng(G + n)
    for mode, workers in MODES[:2]:
        if mode == cq.PARTITION_STATIC and G < 1024:
            workers = G
        p = Pair(G, 700, mode, workers)
        for b in range(3):
            k = (rng.zipf(1.2, n) % G).astype(np.int32)
            v = rng.integers(-10**6, 10**6, n).astype(np.int32)
            p.step(k, v, f"G={G} n={n} batch {b} mode {mode}")
        p.close()


def test_telemetry_records():
    """Kernel-time, worker and phase telemetry describe the last batch and
    do not change its results."""
    note("case: telemetry")
    cfg = skew(1.5, batches=3)
    k, v = host_batch(cfg, 0)
    p = Pair(cfg.groups, cfg.window)
    p.q.set_telemetry(cq.TELEMETRY_KERNEL_TIMES | cq.TELEMETRY_WORKERS | cq.TELEMETRY_PHASES)
    p.step(k, v, "telemetry batch")
    kt = p.q.kernel_times()
    for kind in ("hist", "pass", "update"):
        ms, launches = kt[kind]
        assert launches == 1 and 0 < ms < 100, (kind, ms, launches)
    rec = p.q.worker_trace()
    assert len(rec) >= 1
    plan = p.q.batch_plan()
    # every tuple is handled by exactly one workgroup: light tuples fully,
    # heavy groups through at most W survivors
    worked = [r for r in rec if r[5] > 0]
    assert len(worked) == plan["buckets"]
    assert all(r[3] >= r[2] > 0 for r in worked)
    ph = p.q.phase_trace(1)
    started = [r for r in ph if r[0] > 0]
    assert len(started) == (len(k) + 4095) // 4096
    assert all(r[4] >= r[0] for r in started)
    p.q.set_telemetry(0)
    k2, v2 = host_batch(cfg, 1)
    p.step(k2, v2, "after telemetry")
    p.close()
