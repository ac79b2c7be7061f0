"""Benchmark: sliding-window group-by over Zipf-skewed streams on one MI355X.

Workload (one "step" = one batch through the whole per-batch path: histogram,
plan, scatter, per-group update, emit): 10,000 groups, window W=1000,
batches of 1,048,576 int32 (key, value) tuples, keys Zipf(s) over
[0, 10000) with hot ranks randomly permuted, values uniform in [0, 1e6).
All batches are generated on the device and resident in HBM before timing.

Reported: tuples/s and algorithmic HBM GB/s for s in {0, 0.5, 1, 1.5, 2},
balanced vs static partition, p50/p99 batch latency, and the imbalance of
the per-group phase (per-CU busy-time spread, per-workgroup tuple loads).
The headline value is s=1.5, balanced, with the batches pushed up to
twenty per cq_push_batches call (--per-call; the timed batches are cut
into calls of near-equal size): every batch's results are emitted into its
own buffers, and a call's batches share one set of launches.  The same
batches one cq_push_batch_results call each are reported beside it, and the
static partition runs one batch per call.  Throughput, batch latency (an
event pair per call: a batch's results are complete when its call's work
is) and kernel durations (the library's per-launch events) come from
separate runs over the same batches, because events are stream markers
with idle time of their own.  The roofline object is for the
longest-running kernel of the headline run (one launch processes one
call's batches), beside the end-to-end fraction (algorithmic bytes over
the whole time per batch); its `traffic` is the HBM bytes per launch
from rocprofv3 counters recorded in profiles/traffic_<kind>.md (bytes per
batch there, times this run's batches per launch), or null when that
record was taken on other kernel sources; the whole path's
counter bytes per batch (every launch's record) stand beside the
algorithmic bytes.  The
cpu_baseline is the CPU oracle timed on a bounded sample of the same
headline batches (one thread; a second figure with one thread per host
core up to 16).

Algorithmic bytes per batch (what the method must move): every key and value
read once (8 B per tuple), and per touched group the surviving tuples
written to its ring (4 B each), the evicted values read (4 B each, only
while a group's batch is shorter than its window), its state read and
written (32 B) and its result emitted (24 B).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Window-element additions per second the vector ALUs can issue: the
# from-scratch rescans add one binary64 value per window element (exact for
# these integer sums), and MI355X issues 256 CUs x 64 lanes x 2.4 GHz fp64
# adds (its 78.6 TFLOP/s fp64 vector peak counts an FMA as two).
FP64_ADD_PEAK = 256 * 64 * 2.4e9
SWEEP = (0.0, 0.5, 1.0, 1.5, 2.0)
HEADLINE_S = 1.5
STAGED = 200   # distinct device-resident batches per setting, cycled
METRIC = "tuples/sec and HBM GB/s at Zipf s=0..2, balanced vs static; p99 batch latency"


def algorithmic_bytes(torch, keys_list, groups, window, n):
    """Exact algorithmic bytes of each batch (list), from the batch's key
    histogram and the window fill before it."""
    dev = keys_list[0].device
    cnt = torch.zeros(groups, dtype=torch.int64, device=dev)
    out = []
    for keys in keys_list:
        k = torch.bincount(keys.to(torch.int64), minlength=groups)
        touched = k > 0
        m = torch.minimum(k, torch.tensor(window, device=dev))
        e = torch.where(k < window, torch.clamp(cnt + k - window, min=0), torch.zeros_like(k))
        per_group = (4 * m + 4 * e + 32 + 24) * touched
        out.append(8 * n + int(per_group.sum().item()))
        cnt = torch.minimum(cnt + k, torch.tensor(window, device=dev))
    return out


def run_mode(torch, cq, batches, cfg, mode, warmup, steps, kind="clean", per_call=1):
    """Warm up, then run `steps` batches (push + emit of every batch) with
    no host syncs in between, on a fresh query: one cq_push_batch_results
    call per batch (per_call 1) or cq_push_batches calls of per_call
    batches each, every batch's results into its own buffers.  kind
    "clean": nothing but the batches is enqueued (the throughput figure);
    "latency": an event pair around every call (a batch's results are
    complete when its call's work is, so with several batches per call the
    call's latency is each of its batches' latency); "kernels": the
    library's per-launch event timing.  Events are markers in the stream
    and cost idle time of their own, so each kind is a separate run."""
    dev = batches[0][0].device
    q = cq.Query(cfg.groups, cfg.window, partition=mode)
    cap = min(cfg.groups, cfg.batch)

    def outs_():
        return (torch.empty(cap, dtype=torch.int32, device=dev),
                torch.empty(cap, dtype=torch.int64, device=dev),
                torch.empty(cap, dtype=torch.int32, device=dev),
                torch.empty(cap, dtype=torch.float64, device=dev),
                torch.empty(1, dtype=torch.int64, device=dev))
    outs = [outs_() for _ in range(per_call)]

    def push(i0, i1):
        if per_call == 1:
            for i in range(i0, i1):
                q.push_results_into(*batches[i], *outs[0])
        else:
            q.push_batches_into(batches[i0:i1], outs[:i1 - i0])

    def cut(a, z):  # [a, z) in ceil((z - a) / per_call) calls of near-equal size
        n = z - a
        k = -(-n // per_call)
        edges = [a + (n * c) // k for c in range(k + 1)]
        return list(zip(edges[:-1], edges[1:]))

    for i0, i1 in cut(0, warmup):
        push(i0, i1)
    torch.cuda.synchronize()
    if kind == "kernels":
        q.set_telemetry(cq.TELEMETRY_KERNEL_TIMES)
        q.kernel_times()
    res = {}
    calls = cut(warmup, warmup + steps)
    if kind == "latency":
        starts = [torch.cuda.Event(enable_timing=True) for _ in calls]
        ends = [torch.cuda.Event(enable_timing=True) for _ in calls]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, (i0, i1) in enumerate(calls):
        if kind == "latency":
            starts[c].record()
        push(i0, i1)
        if kind == "latency":
            ends[c].record()
    torch.cuda.synchronize()
    res["wall_s"] = time.perf_counter() - t0
    if kind == "latency":
        res["lat_ms"] = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    if kind == "kernels":
        res["kernels"] = q.kernel_times()
        q.set_telemetry(0)
    res["plan"] = q.batch_plan()
    q.close()
    return res


def techniques(torch, cq, s_list, warmup, steps):
    """The Section 5 comparison: no balancing (the static ranges), the six
    Section 4 techniques on the same 1024 static workers (host step after
    every batch, one batch of delay, threshold 1000, pot 0.5), and the
    device-side balanced partition, on DS2-like (hot keys are the smallest
    ids) and DS3-like (permuted) Zipf streams of 10,000 groups, W=1000,
    1,048,576-tuple batches."""
    from workloads import DeviceStream, skew
    dev = torch.device("cuda", 0)
    modes = [(cq.PARTITION_STATIC, "no balance (static)")]
    modes += [(m, nm) for nm, m in cq.POLICIES.items()]
    modes += [(cq.PARTITION_BALANCED, "balanced (device)")]
    rows = []
    for s in s_list:
        for permuted, ds in ((False, "DS2-like"), (True, "DS3-like")):
            cfg = skew(s, permuted=permuted, batches=warmup + steps)
            stream = DeviceStream(cfg, dev)
            batches = [stream.batch(b) for b in range(warmup + steps)]
            torch.cuda.synchronize()
            base = None
            for mode, name in modes:
                q = cq.Query(cfg.groups, cfg.window, partition=mode)
                for b in range(warmup):
                    q.push(*batches[b])
                torch.cuda.synchronize()
                moves0 = q.policy_stats()[3]
                t0 = time.perf_counter()
                for b in range(warmup, warmup + steps):
                    q.push(*batches[b])
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                st = q.policy_stats()
                q.close()
                ms = 1e3 * wall / steps
                base = ms if base is None else base
                row = {"dataset": f"{ds} s={s:g}", "partition": name,
                       "ms_per_batch": round(ms, 4),
                       "tuples_per_s": steps * cfg.batch / wall,
                       "time_vs_no_balance": round(ms / base, 4)}
                if mode >= cq.PARTITION_GETFIRST:
                    row["moves_timed"] = st[3] - moves0
                    row["last_batch_tpt_max_min"] = [st[1], st[2]]
                rows.append(row)
                print(json.dumps({"progress": row}), file=sys.stderr, flush=True)
            del batches, stream
            torch.cuda.empty_cache()
    return rows


def per_tuple(torch, cq, batches, cfg, warmup, steps, passes_list):
    """The paper-literal variant (cq_push_batch_tuples): per-tuple window
    SUM/COUNT/AVG after every insertion, incrementally (passes 0) or with
    every window summed from scratch (passes 1 and 10, Section 5.1 and the
    ten-fold scan of Section 5.2).  Whole pushes timed on the device stream,
    then the k_tuples launches alone with the library's events."""
    dev = batches[0][0].device
    n = cfg.batch
    sums = torch.empty(n, dtype=torch.int64, device=dev)
    counts = torch.empty(n, dtype=torch.int32, device=dev)
    avgs = torch.empty(n, dtype=torch.float64, device=dev)
    rows = []
    for passes in passes_list:
        st = steps if passes <= 1 else max(4, steps // 4)
        q = cq.Query(cfg.groups, cfg.window)
        for b in range(warmup):
            q.push_tuples_into(*batches[b], sums, counts, avgs, passes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(warmup, warmup + st):
            q.push_tuples_into(*batches[b], sums, counts, avgs, passes)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        q.set_telemetry(cq.TELEMETRY_KERNEL_TIMES)
        q.kernel_times()
        for b in range(warmup, warmup + st):
            q.push_tuples_into(*batches[b], sums, counts, avgs, passes)
        kt = q.kernel_times()
        q.close()
        ms_t, launches = kt["tuples"]
        k_us = 1e3 * ms_t / max(1, launches)
        row = {"passes": passes, "ms_per_batch": round(1e3 * wall / st, 4),
               "tuples_per_s": st * n / wall, "k_tuples_avg_us": round(k_us, 2),
               "output_bytes_per_batch": 20 * n}
        if passes:
            # window elements summed per launch: every tuple's W entries, each pass
            adds = float(n) * cfg.window * passes
            row["window_elems_per_s"] = adds / (k_us * 1e-6)
            row["alu_frac"] = round(row["window_elems_per_s"] / FP64_ADD_PEAK, 4)
        rows.append(row)
        print(json.dumps({"progress": {"per_tuple": row}}), file=sys.stderr, flush=True)
    return rows


def paper_shape_rows(torch, cq, warmup, steps, tuple_passes):
    """Tables 1 and 2 and the ten-fold scan at the paper's own setting
    (Section 5.1): 40,000 groups, W=100, 50,000-tuple batches.  On DS1-,
    DS2- and DS3-like streams: no balancing (the static ranges), the six
    Section 4 techniques (threshold 1000, pot 0.5, host step after every
    batch) on 1,024 static workers (the paper's grid of 4 blocks of 256
    threads) and on 4,096 (the most a static partition takes: the analogue
    of its grid of 64 blocks, 16,384 threads), and the device-side balanced
    partition; then the per-tuple form (rescan after every insertion, once
    and ten times) on DS2 and DS3.  Whole pushes timed on the host clock
    around a device synchronisation."""
    from workloads import host_batch, paper_shape
    dev = torch.device("cuda", 0)
    rows, tuples = [], []
    for dataset in ("DS1", "DS2", "DS3"):
        cfg = paper_shape(dataset)
        batches = []
        for b in range(warmup + steps):
            k, v = host_batch(cfg, b)
            batches.append((torch.from_numpy(k).to(dev), torch.from_numpy(v).to(dev)))
        torch.cuda.synchronize()
        for workers in (1024, 4096):
            modes = [(cq.PARTITION_STATIC, "no balance (static)")]
            modes += [(m, nm) for nm, m in cq.POLICIES.items()]
            if workers == 1024:
                modes += [(cq.PARTITION_BALANCED, "balanced (device)")]
            base = None
            for mode, name in modes:
                q = cq.Query(cfg.groups, cfg.window)
                q.set_policy_params(1000, 0.5)
                q.set_partition(mode, workers if mode != cq.PARTITION_BALANCED else 0)
                for b in range(warmup):
                    q.push(*batches[b])
                torch.cuda.synchronize()
                moves0 = q.policy_stats()[3]
                t0 = time.perf_counter()
                for b in range(warmup, warmup + steps):
                    q.push(*batches[b])
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                st = q.policy_stats()
                q.close()
                ms = 1e3 * wall / steps
                base = ms if base is None else base
                row = {"dataset": dataset, "workers": workers if mode != cq.PARTITION_BALANCED
                       else None, "partition": name, "ms_per_batch": round(ms, 4),
                       "tuples_per_s": steps * cfg.batch / wall,
                       "time_vs_no_balance": round(ms / base, 4)}
                if mode >= cq.PARTITION_GETFIRST:
                    row["moves_timed"] = st[3] - moves0
                    row["last_batch_tpt_max_min"] = [st[1], st[2]]
                rows.append(row)
                print(json.dumps({"progress": {"paper_shape": row}}), file=sys.stderr, flush=True)
        if dataset != "DS1" and tuple_passes:
            for r in per_tuple(torch, cq, batches, cfg, warmup, steps, tuple_passes):
                r["dataset"] = dataset
                tuples.append(r)
        del batches
    return {"groups": 40_000, "window": 100, "batch": 50_000, "zipf_s": 1.0,
            "threshold": 1000, "pot": 0.5, "partitions": rows, "per_tuple": tuples}


def serving(torch, cq, lambdas, seconds, lanes=8, slots=2, nq=256):
    """The serving loop (cq_server_*): `nq` resident queries (groups
    log-uniform in [100, 1e6], windows in [10, 1e4]) admitted by device
    footprint against 80% of the free HBM; batches (lognormal sizes, median
    65,536, Zipf s=1.5 keys whose hot set is redrawn every 10 s of arrival
    time) arrive as a Poisson process at each rate in `lambdas` for
    `seconds`, each for a query drawn uniformly; latency is submission to
    completion."""
    from workloads import ServingBatches, serving_queries, serving_sizes
    dev = torch.device("cuda", 0)
    torch.cuda.empty_cache()
    qs = serving_queries(nq)
    epochs = int(len(lambdas) * seconds // 10) + 1
    per = 2  # batches per query and epoch
    sizes = serving_sizes(nq * epochs * per, 0).reshape(nq, epochs, per)
    gen = ServingBatches(dev)
    t0 = time.perf_counter()
    batches = [[[gen.batch(q, G, e, i, int(sizes[q, e, i])) for i in range(per)]
                for e in range(epochs)] for q, (G, _) in enumerate(qs)]
    outs = []
    for q, (G, _) in enumerate(qs):
        cap = int(max(1, min(G, sizes[q].max())))
        outs.append((torch.empty(cap, dtype=torch.int32, device=dev),
                     torch.empty(cap, dtype=torch.int64, device=dev),
                     torch.empty(cap, dtype=torch.int32, device=dev),
                     torch.empty(cap, dtype=torch.float64, device=dev),
                     torch.empty(1, dtype=torch.int64, device=dev)))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    srv = cq.Server(0, lanes, slots)
    admitted, rejected = [], 0
    t0 = time.perf_counter()
    for q, (G, W) in enumerate(qs):
        try:
            admitted.append((q, srv.add_query(G, W)))
        except cq.CQError as e:
            if e.code != cq.ERR_OOM:
                raise
            rejected += 1
    setup_s = time.perf_counter() - t0
    held = srv.stats()
    rows = []
    arrival0 = 0.0
    for lam in lambdas:
        rng = np.random.default_rng([20130909, 81, int(lam)])
        srv.stats()
        t, start, count, tuples = 0.0, time.perf_counter(), 0, 0
        while True:
            t += rng.exponential(1.0 / lam)
            if t >= seconds:
                break
            wait_s = t - (time.perf_counter() - start)
            if wait_s > 0:
                time.sleep(wait_s)
            q, qid = admitted[int(rng.integers(len(admitted)))]
            e = min(epochs - 1, int((arrival0 + t) // 10))
            k, v = batches[q][e][int(rng.integers(per))]
            srv.submit(qid, k, v, *outs[q])
            count += 1
            tuples += k.numel()
        srv.wait()
        st = srv.stats()
        arrival0 += seconds
        row = {"arrivals_per_s": lam, "requests": int(st["requests"]),
               "p50_ms": round(st["p50_us"] / 1e3, 4), "p99_ms": round(st["p99_us"] / 1e3, 4),
               "max_ms": round(st["max_us"] / 1e3, 4), "tuples_per_s": st["tuples_per_s"],
               "mean_batch": round(tuples / max(1, count))}
        rows.append(row)
        print(json.dumps({"progress": {"serving": row}}), file=sys.stderr, flush=True)
    # capacity: the same mix submitted as fast as the client can, for as
    # many requests as the highest rate delivered
    rng = np.random.default_rng([20130909, 82])
    burst = max(1, rows[-1]["requests"]) if rows else 1000
    srv.stats()
    tuples = 0
    for _ in range(burst):
        q, qid = admitted[int(rng.integers(len(admitted)))]
        k, v = batches[q][epochs - 1][int(rng.integers(per))]
        srv.submit(qid, k, v, *outs[q])
        tuples += k.numel()
    srv.wait()
    st = srv.stats()
    sat = {"requests": int(st["requests"]), "p50_ms": round(st["p50_us"] / 1e3, 4),
           "p99_ms": round(st["p99_us"] / 1e3, 4), "tuples_per_s": st["tuples_per_s"],
           "mean_batch": round(tuples / burst)}
    print(json.dumps({"progress": {"serving_saturated": sat}}), file=sys.stderr, flush=True)
    srv.close()
    return {"queries": nq, "admitted": len(admitted), "rejected_by_footprint": rejected,
            "bytes_held": int(held["bytes_held"]), "budget": int(held["budget"]),
            "lanes": lanes, "slots_per_lane": slots, "seconds_per_rate": seconds,
            "setup_s": round(setup_s, 2), "generation_s": round(gen_s, 2), "rates": rows,
            "saturated": sat}


def drifting_run(torch, cq, warmup, steps):
    """The large stream: 1,048,576 groups, W=100, 16,777,216-tuple Zipf
    s=1.2 batches, hot permutation redrawn every 50 batches (the timed
    batches straddle a redraw).  Balanced partition, push + emit, timed on
    the device stream; algorithmic bytes per batch as for the headline."""
    from workloads import DeviceStream, drifting
    dev = torch.device("cuda", 0)
    torch.cuda.empty_cache()
    cfg = drifting(batches=60)
    first = 50 - warmup - steps // 2  # so that the redraw at batch 50 is inside
    ds = DeviceStream(cfg, dev)
    idx = list(range(first, first + warmup + steps))
    batches = [ds.batch(b) for b in idx]
    torch.cuda.synchronize()
    bytes_per = algorithmic_bytes(torch, [k for k, _ in batches], cfg.groups, cfg.window,
                                  cfg.batch)
    q = cq.Query(cfg.groups, cfg.window)
    cap = min(cfg.groups, cfg.batch)
    outs = (torch.empty(cap, dtype=torch.int32, device=dev),
            torch.empty(cap, dtype=torch.int64, device=dev),
            torch.empty(cap, dtype=torch.int32, device=dev),
            torch.empty(cap, dtype=torch.float64, device=dev),
            torch.empty(1, dtype=torch.int64, device=dev))
    for b in range(warmup):
        q.push_results_into(*batches[b], *outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(warmup, warmup + steps):
        q.push_results_into(*batches[b], *outs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan = q.batch_plan()
    q.close()
    alg = sum(bytes_per[warmup:])
    out = {"workload": cfg.name, "batches_timed": steps, "first_batch": idx[warmup],
           "ms_per_batch": round(1e3 * wall / steps, 3),
           "tuples_per_s": steps * cfg.batch / wall,
           "alg_MB_per_batch": round(alg / steps / 1e6, 2),
           "alg_GBps": alg / wall / 1e9, "alg_frac_of_hbm": round(alg / wall / 1e9 / HBM_PEAK_GBS, 4),
           "heavy_groups_last": int(plan["heavy_groups"]), "touched_last": int(plan["touched"])}
    print(json.dumps({"progress": {"drifting": out}}), file=sys.stderr, flush=True)
    del batches
    torch.cuda.empty_cache()
    return out


def multi(torch, cq, nq=64, warmup=2, steps=6, lanes=8, reps=2):
    """The multi-query set (cq_multi_*): `nq` queries (groups and windows
    log-uniform) share 4,194,304-tuple Zipf s=1.0 batches, each taking key
    mod its group count.  Timed: every query on one lane, the queries spread
    over `lanes` lanes, the same after the autotuner's window, and that set
    replayed as one captured HIP graph per batch."""
    from workloads import DeviceStream, multi_queries, multi_stream
    dev = torch.device("cuda", 0)
    torch.cuda.empty_cache()
    spec = multi_queries(nq)
    ncand = 3
    total = warmup + 4 * steps + ncand * reps + 1
    cfg = multi_stream(batches=total)
    ds = DeviceStream(cfg, dev)
    batches = [ds.batch(b) for b in range(total)]
    qs = []
    for G, W in spec:
        q = cq.Query(G, W)
        q.set_key_mod(True)
        qs.append(q)
    ring_bytes = sum(4 * G * W for G, W in spec)
    it = iter(batches)

    def timed(m, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            m.push(*next(it))
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    rows = {}
    m1 = cq.Multi(qs, 1)
    for _ in range(warmup):
        m1.push(*next(it))
    rows["one_lane"] = timed(m1, steps)
    m1.close()
    m = cq.Multi(qs, lanes)
    rows[f"{lanes}_lanes"] = timed(m, steps)
    m.tune(reps)
    for _ in range(ncand * reps):
        m.push(*next(it))
    rows[f"{lanes}_lanes_tuned"] = timed(m, steps)
    m.set_graph(True)
    m.push(*next(it))  # captures this batch size's graph
    rows[f"{lanes}_lanes_tuned_graph"] = timed(m, steps)
    plan = m.plan()
    m.close()
    for q in qs:
        q.close()
    out = {"queries": nq, "batch": cfg.batch, "ring_bytes": ring_bytes, "lanes": lanes,
           "timed_batches": steps}
    for k, sec in rows.items():
        out[k] = {"ms_per_batch": round(1e3 * sec, 3), "input_tuples_per_s": cfg.batch / sec,
                  "query_tuples_per_s": nq * cfg.batch / sec}
    out["tuned_modes"] = {
        "balanced": sum(p["mode"] == cq.PARTITION_BALANCED for p in plan),
        "static_1024": sum(p["mode"] == cq.PARTITION_STATIC and p["workers"] == 1024 for p in plan),
        "static_4096": sum(p["mode"] == cq.PARTITION_STATIC and p["workers"] == 4096 for p in plan)}
    print(json.dumps({"progress": {"multi": out}}), file=sys.stderr, flush=True)
    return out


def imbalance(torch, cq, batches, cfg, mode, warmup=3):
    """Per-CU busy time of the per-group phase on one batch (after `warmup`
    batches): the union of the device-clock intervals of the workgroups that
    ran on each compute unit (XCC, shader engine, array, CU from the HW_ID
    register), over the CUs that did work.  Also the per-workgroup tuple
    loads (the paper's per-worker tuple counts)."""
    warmup = max(0, min(warmup, len(batches) - 1))
    q = cq.Query(cfg.groups, cfg.window, partition=mode)
    for b in range(warmup):
        q.push(*batches[b])
    q.set_telemetry(cq.TELEMETRY_WORKERS)
    q.push(*batches[warmup])
    rec = q.worker_trace()
    q.set_telemetry(0)
    q.close()
    t_first = min(r[2] for r in rec)
    per_cu = {}
    for hw, xcc, t0, t1, tuples, items in rec:
        if tuples <= 0:
            continue
        cu = (xcc, (hw >> 13) & 7, (hw >> 12) & 1, (hw >> 8) & 15)
        per_cu.setdefault(cu, []).append((t0, t1))
    busy = []
    for iv in per_cu.values():
        iv.sort()
        tot, cs, ce = 0, iv[0][0], iv[0][1]
        for a, b in iv[1:]:
            if a > ce:
                tot += ce - cs
                cs, ce = a, b
            else:
                ce = max(ce, b)
        busy.append((tot + ce - cs) * 0.01)  # 100 MHz ticks -> us
    loads = [r[4] for r in rec if r[4] > 0]
    busy = np.array(busy)
    span = (max(r[3] for r in rec) - t_first) * 0.01
    return {"cus_with_work": int(len(busy)),
            "cu_busy_max_us": round(float(busy.max()), 2),
            "cu_busy_mean_us": round(float(busy.mean()), 2),
            "cu_busy_max_over_mean": round(float(busy.max() / busy.mean()), 3),
            "cu_busy_cv": round(float(busy.std() / busy.mean()), 3),
            "phase_span_us": round(span, 2),
            "wg_tuples_max_over_mean": round(float(max(loads) / np.mean(loads)), 3)}


KERNEL_SOURCES = [os.path.join(ROOT, "paper_1309_0634_amd", "csrc", f)
                  for f in ("cq_kernels.hip", "cq_device.h", "cq_internal.h")]
PROFILES = os.path.join(ROOT, "profiles")


def measured_traffic(kernel: str):
    """HBM bytes per batch of `kernel` (its bytes per launch over the batches
    each recorded launch processed), recorded from rocprofv3 FETCH_SIZE and
    WRITE_SIZE counters in profiles/traffic_<kernel>.md, or None when that
    record was taken on a different kernel source than the one built now."""
    path = os.path.join(PROFILES, f"traffic_{kernel}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    m_n = re.search(r"batches_per_launch:\s*([0-9]+)", text)
    if not (m_sha and m_b and m_n):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:  # the kernels' source and the headers they build on
        h.update(open(f, "rb").read())
    sha = h.hexdigest()
    return float(m_b.group(1)) / int(m_n.group(1)) if sha == m_sha.group(1) else None


def copy_calibration(torch, mib: int):
    """One plain device-to-device copy of `mib` MiB, so that a profiler run
    of this command also shows what the traffic counters read for a kernel
    of known size."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batches_host, cfg, budget_s, threads=1):
    """The CPU oracle over the headline batches (cycled, continuing one
    stream) until about `budget_s` seconds of work.  Returns (batches, s)."""
    from oracle import RingOracle
    ora = RingOracle(cfg.groups, cfg.window, threads=threads)
    done, t = 0, 0.0
    while t < budget_s:
        for k, v in batches_host:
            t0 = time.perf_counter()
            ora.push(k, v)
            t += time.perf_counter() - t0
            done += 1
            if t >= budget_s:
                break
    ora.close()
    return done, t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of CPU-oracle work for the cpu_baseline sample")
    ap.add_argument("--sweep", default=",".join(str(s) for s in SWEEP))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--modes", default="balanced,static",
                    help="partitions to run (the headline needs balanced)")
    ap.add_argument("--techniques", default="1.0,1.5",
                    help="Zipf s values of the Section 4 technique comparison ('' skips it)")
    ap.add_argument("--tech-steps", type=int, default=40)
    ap.add_argument("--tuple-passes", default="0,1,10",
                    help="passes of the per-tuple variant to time ('' skips it)")
    ap.add_argument("--paper-steps", type=int, default=40,
                    help="timed batches per row at the paper's setting (0 skips it)")
    ap.add_argument("--drift", type=int, default=6,
                    help="timed batches of the large drifting stream (0 skips it)")
    ap.add_argument("--multi", type=int, default=64,
                    help="queries of the multi-query set (0 skips it)")
    ap.add_argument("--serving", default="10,50,100,250,500",
                    help="arrival rates (batches/s) of the serving loop ('' skips it)")
    ap.add_argument("--serving-seconds", type=float, default=3.0)
    ap.add_argument("--per-call", type=int, default=20,
                    help="batches per cq_push_batches call of the balanced partition "
                         "(20: one set of the library's launches, CQ_CHAIN_BATCHES)")
    ap.add_argument("--calibrate", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
              "(on several GPUs the path would shard groups by owner and exchange each "
              "group's last W tuples of a batch in one all-to-all)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1309_0634_amd as cq
    from workloads import DeviceStream, skew

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.calibrate:
        copy_calibration(torch, args.calibrate)
    sweep = [float(x) for x in args.sweep.split(",")]
    rows = []
    headline = None
    for s in sweep:
        cfg = skew(s)
        ds = DeviceStream(cfg, dev)
        # STAGED distinct batches (1.6 GiB, several times the 256 MB
        # last-level cache), cycled: warm-up and timed pushes never find the
        # inputs of a recent batch still cached, whatever --steps is
        staged = [ds.batch(b) for b in range(STAGED)]
        batches = [staged[i % STAGED] for i in range(args.warmup + args.steps)]
        del staged
        torch.cuda.synchronize()
        bytes_per = algorithmic_bytes(torch, [k for k, _ in batches], cfg.groups, cfg.window,
                                      cfg.batch)
        timed_bytes = sum(bytes_per[args.warmup:])
        modes = [(m, nm) for m, nm in ((cq.PARTITION_BALANCED, "balanced"),
                                        (cq.PARTITION_STATIC, "static"))
                 if nm in args.modes.split(",")]
        for mode, name in modes:
            is_head = (s == HEADLINE_S and mode == cq.PARTITION_BALANCED)
            # the balanced partition runs PER_CALL batches per cq_push_batches
            # call (every batch's results emitted); the static baseline one
            # batch per call
            pc = args.per_call if mode == cq.PARTITION_BALANCED else 1
            r = run_mode(torch, cq, batches, cfg, mode, args.warmup, args.steps, per_call=pc)
            lat = run_mode(torch, cq, batches, cfg, mode, args.warmup, args.steps, "latency",
                           per_call=pc)
            tuples = args.steps * cfg.batch
            row = {
                "s": s, "partition": name, "batches_per_call": pc,
                "tuples_per_s": tuples / r["wall_s"],
                "alg_GBps": timed_bytes / r["wall_s"] / 1e9,
                "ms_per_batch": 1e3 * r["wall_s"] / args.steps,
                "p50_batch_ms": float(np.percentile(lat["lat_ms"], 50)),
                "p99_batch_ms": float(np.percentile(lat["lat_ms"], 99)),
                "alg_MB_per_batch": timed_bytes / args.steps / 1e6,
                "heavy_groups": int(r["plan"]["heavy_groups"]),
                "buckets": int(r["plan"]["buckets"]),
                "touched": int(r["plan"]["touched"]),
                "imbalance": imbalance(torch, cq, batches, cfg, mode),
            }
            if pc > 1:  # the same batches one call each, for comparison
                r1 = run_mode(torch, cq, batches, cfg, mode, args.warmup, args.steps)
                l1 = run_mode(torch, cq, batches, cfg, mode, args.warmup, args.steps, "latency")
                row["one_batch_per_call"] = {
                    "tuples_per_s": tuples / r1["wall_s"],
                    "ms_per_batch": 1e3 * r1["wall_s"] / args.steps,
                    "p50_batch_ms": float(np.percentile(l1["lat_ms"], 50)),
                    "p99_batch_ms": float(np.percentile(l1["lat_ms"], 99))}
            rows.append(row)
            print(json.dumps({"progress": row}), file=sys.stderr, flush=True)
            if is_head:
                kr = run_mode(torch, cq, batches, cfg, mode, args.warmup, args.steps, "kernels",
                              per_call=pc)
                r["kernels"] = kr["kernels"]
                headline = (row, r, timed_bytes, cfg, batches)
        if not (s == HEADLINE_S):
            del batches
            torch.cuda.empty_cache()

    if headline is None:
        print("bench.py: the sweep must include s=1.5", file=sys.stderr)
        sys.exit(2)
    row, r, timed_bytes, cfg, batches = headline
    headline = None
    kern = {k: v for k, v in r["kernels"].items() if v[1] > 0}
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms, dom_launches = kern[dom]
    avg_bytes = timed_bytes / args.steps
    # one launch of each kernel processes one call's batches
    per_call = args.steps / dom_launches
    per_launch = avg_bytes * per_call
    achieved = per_launch / (dom_ms / dom_launches * 1e-3) / 1e9
    traffic = measured_traffic(dom)
    traffic = None if traffic is None else round(traffic * per_call)
    e2e = avg_bytes / (row["ms_per_batch"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "kernel_avg_us": round(1e3 * dom_ms / dom_launches, 2),
                "batches_per_launch": round(per_call, 3),
                "alg_bytes_per_launch": round(per_launch),
                "end_to_end_GBps": round(e2e, 1),
                "end_to_end_frac": round(e2e / HBM_PEAK_GBS, 4),
                "kernel_times_ms": {k: round(v[0], 3) for k, v in kern.items()},
                "kernel_launches": {k: v[1] for k, v in kern.items()}}
    # the whole path's counter bytes (every kind's record, per batch), when
    # every record matches the kernels built now
    recs = [measured_traffic(k) for k in kern]
    if all(t is not None for t in recs):
        path_b = sum(recs)
        roofline["path_traffic_bytes_per_batch"] = round(path_b)
        roofline["alg_bytes_per_batch"] = round(avg_bytes)
        roofline["path_traffic_over_alg"] = round(path_b / avg_bytes, 3)
    else:
        roofline["path_traffic_bytes_per_batch"] = None
    pt = None
    if args.tuple_passes:
        pt = per_tuple(torch, cq, batches, cfg, min(args.warmup, 5), min(args.steps, 40),
                       [int(x) for x in args.tuple_passes.split(",")])
    host = None if args.no_cpu else [(k.cpu().numpy(), v.cpu().numpy())
                                     for k, v in batches[:STAGED]]
    del batches
    torch.cuda.empty_cache()
    tech = None
    if args.techniques:
        tech = techniques(torch, cq, [float(x) for x in args.techniques.split(",")],
                          min(args.warmup, 5), args.tech_steps)
    paper = None
    if args.paper_steps:
        paper = paper_shape_rows(torch, cq, 5, args.paper_steps,
                                 [int(x) for x in args.tuple_passes.split(",")]
                                 if args.tuple_passes else [])
    drift = drifting_run(torch, cq, 2, args.drift) if args.drift else None
    mq = multi(torch, cq, args.multi) if args.multi else None
    serve = None
    if args.serving:
        serve = serving(torch, cq, [float(x) for x in args.serving.split(",")],
                        args.serving_seconds)
    cpu = cpu_mt = None
    if not args.no_cpu:
        done, t = cpu_baseline(host, cfg, args.cpu_budget)
        cpu = {"value": done * cfg.batch / t, "unit": "tuples/s", "cores": 1, "kind": "oracle",
               "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
               "sample": f"{done} batches of the s=1.5 stream (the {len(host)} headline batches "
                         f"of 1,048,576 tuples, cycled), C oracle, one thread, {t:.1f} s"}
        nthreads = min(16, os.cpu_count() or 1)
        done, t = cpu_baseline(host, cfg, args.cpu_budget / 2, threads=nthreads)
        cpu_mt = {"value": done * cfg.batch / t, "unit": "tuples/s", "cores": nthreads,
                  "kind": "oracle",
                  "sample": f"{done} batches of the same stream, C oracle with {nthreads} threads "
                            f"(each owns a key range), {t:.1f} s"}
    out = {
        "metric": METRIC,
        "value": row["tuples_per_s"],
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": row["ms_per_batch"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "zipf_skew_g10000_w1000_n1048576_s1.5_balanced",
                   "groups": cfg.groups, "window": cfg.window, "batch": cfg.batch,
                   "zipf_s": HEADLINE_S, "partition": "balanced",
                   "batches_per_call": row["batches_per_call"], "parallelism": "1gpu"},
        "alg_GBps": row["alg_GBps"],
        "one_batch_per_call": row.get("one_batch_per_call"),
        "p50_batch_ms": row["p50_batch_ms"],
        "p99_batch_ms": row["p99_batch_ms"],
        "imbalance_s1.5": {r["partition"]: r["imbalance"] for r in rows if r["s"] == HEADLINE_S},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_all_threads": cpu_mt,
        "sweep": rows,
        "techniques": tech,
        "per_tuple": pt,
        "paper_shape": paper,
        "drifting": drift,
        "multi_query": mq,
        "serving": serve,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
