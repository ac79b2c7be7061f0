"""Python binding of libcq (include/cq.h): sliding-window group-by on MI355X.

Argument marshalling only.  Every step of the update runs in the HIP
kernels of ``libcq.so``; torch tensors are used for device memory and the
stream handle.  The binding fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(PKG, "libcq.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "cq.h")

SUM, COUNT, AVG = 1, 2, 4
OK, ERR_INVALID, ERR_OOM, ERR_KEY_RANGE, ERR_HIP = 0, -1, -2, -3, -4
PARTITION_BALANCED, PARTITION_STATIC = 0, 1
# the Section 4 techniques, on the static workers
(PARTITION_GETFIRST, PARTITION_CHECKALL, PARTITION_PROBCHECK, PARTITION_BESTBALANCE,
 PARTITION_SHIFT, PARTITION_SHIFTLOCAL) = range(2, 8)
POLICIES = {"getFirst": PARTITION_GETFIRST, "checkAll": PARTITION_CHECKALL,
            "probCheck": PARTITION_PROBCHECK, "bestBalance": PARTITION_BESTBALANCE,
            "shift": PARTITION_SHIFT, "shiftLocal": PARTITION_SHIFTLOCAL}
STATIC_KEYS_MAX = 2048
TELEMETRY_KERNEL_TIMES, TELEMETRY_WORKERS, TELEMETRY_PHASES = 1, 2, 4
KERNEL_KINDS = ("hist", "pass", "update", "emit", "other", "plan", "tuples", "prep", "apply")
TUPLE_MAX_WINDOW = 1024
TUPLE_MAX_PASSES = 64
TUPLE_MAX_GROUPS = 1 << 21
MAX_BATCH = 1 << 30
MAX_WINDOW = (1 << 22) - 1
PIPE_MAX = 1 << 20
CHAIN_BATCHES = 20
NOALLOC_MAX_BATCH = 1 << 18
NOALLOC_MAX_GROUPS = 16384

_lib: Optional[ctypes.CDLL] = None


class CQError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = strerror(code) if _lib is not None else f"status {code}"
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


def lib() -> ctypes.CDLL:
    """The loaded libcq.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch first: its wheel ships a HIP runtime with the same soname as
        # the system one the library links against, so whichever loads first
        # serves the whole process; torch does not start on the other one,
        # and the library runs on torch's (one runtime, shared pointers).
        import torch  # noqa: F401
        if not os.path.exists(LIBRARY):
            raise ImportError(f"{LIBRARY} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIBRARY)
        P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        pi64 = ctypes.POINTER(ctypes.c_int64)
        pdbl = ctypes.POINTER(ctypes.c_double)
        sig = {
            "cq_create": ([i64, i32, u32, ctypes.POINTER(P)], ctypes.c_int),
            "cq_reserve": ([P, i64], ctypes.c_int),
            "cq_set_partition": ([P, i32, i32], ctypes.c_int),
            "cq_push_batch": ([P, P, P, i64, P], ctypes.c_int),
            "cq_results": ([P, P, P, P, P, P, P], ctypes.c_int),
            "cq_push_batch_results": ([P, P, P, i64, P, P, P, P, P, P], ctypes.c_int),
            "cq_push_batch_results_noalloc": ([P, P, P, i64, P, P, P, P, P, P], ctypes.c_int),
            "cq_status": ([P], ctypes.c_int),
            "cq_destroy": ([P], ctypes.c_int),
            "cq_strerror": ([ctypes.c_int], ctypes.c_char_p),
            "cq_set_telemetry": ([P, i32], ctypes.c_int),
            "cq_kernel_times": ([P, pdbl, pi64, i32], ctypes.c_int),
            "cq_worker_trace": ([P, pi64, i64, pi64], ctypes.c_int),
            "cq_batch_plan": ([P, pi64], ctypes.c_int),
            "cq_phase_trace": ([P, i32, pi64, i64, pi64], ctypes.c_int),
            "cq_push_batches": ([P, i32, P, P, P, P, P, P, P, P, P], ctypes.c_int),
            "cq_push_batch_tuples": ([P, P, P, i64, i32, P, P, P, P], ctypes.c_int),
            "cq_set_policy_params": ([P, i64, ctypes.c_double], ctypes.c_int),
            "cq_query_footprint": ([i64, i32], i64),
            "cq_query_groups": ([P, pi64], ctypes.c_int),
            "cq_set_key_mod": ([P, i32], ctypes.c_int),
            "cq_multi_create": ([P, i32, i32, ctypes.POINTER(P)], ctypes.c_int),
            "cq_multi_push": ([P, P, P, i64, P], ctypes.c_int),
            "cq_multi_tune": ([P, i32], ctypes.c_int),
            "cq_multi_plan": ([P, P, P, P, P], ctypes.c_int),
            "cq_multi_destroy": ([P], ctypes.c_int),
            "cq_multi_set_graph": ([P, i32], ctypes.c_int),
            "cq_server_create": ([i64, i32, i32, ctypes.POINTER(P)], ctypes.c_int),
            "cq_server_add_query": ([P, i64, i32, u32, ctypes.POINTER(i32)], ctypes.c_int),
            "cq_server_remove_query": ([P, i32], ctypes.c_int),
            "cq_server_submit": ([P, i32, P, P, i64, P, P, P, P, P, pi64], ctypes.c_int),
            "cq_server_wait": ([P, i64], ctypes.c_int),
            "cq_server_stats": ([P, pdbl], ctypes.c_int),
            "cq_server_destroy": ([P], ctypes.c_int),
            "cq_policy_stats": ([P, pi64], ctypes.c_int),
            "cq_policy_apply": ([i32, i32, i64, P, P, i64, P, P, i64, ctypes.c_double, i32,
                                 pi64], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().cq_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != OK:
        raise CQError(rc, what)


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def policy_apply(policy: int, counts, wstart, wlist, threshold: int = 1000, pot: float = 0.5,
                 max_keys: int = STATIC_KEYS_MAX, keys=None):
    """One host-side balancing step (cq_policy_apply) on numpy arrays: the
    mapping ``wstart``/``wlist`` (int32, CSR, modified in place), the
    batch's per-group ``counts`` (int32) and, for probCheck, the batch's
    ``keys`` in arrival order (int32).  Returns the number of moves."""
    import numpy as np
    arrays = (counts, wstart, wlist) + (() if keys is None else (keys,))
    for a in arrays:
        if not (isinstance(a, np.ndarray) and a.dtype == np.int32 and a.flags.c_contiguous):
            raise TypeError("policy_apply takes C-contiguous int32 numpy arrays")
    if counts.shape[0] != wlist.shape[0]:
        raise ValueError("counts and wlist must both have one entry per group")
    n = 0 if keys is None else int(keys.shape[0])
    moves = ctypes.c_int64(0)
    _check(lib().cq_policy_apply(int(policy), int(wstart.shape[0] - 1), int(wlist.shape[0]),
                                 counts.ctypes.data, keys.ctypes.data if n else None, n,
                                 wstart.ctypes.data, wlist.ctypes.data, int(threshold),
                                 float(pot), int(max_keys), ctypes.byref(moves)),
           "cq_policy_apply")
    return moves.value


class Query:
    """One continuous query: ``groups`` group ids, a ``window``-tuple window
    per group (cq_create)."""

    def __init__(self, groups: int, window: int, aggregates: int = SUM | COUNT | AVG,
                 partition: int = PARTITION_BALANCED, workers: int = 0,
                 reserve: int = 0):
        L = lib()
        h = ctypes.c_void_p()
        _check(L.cq_create(int(groups), int(window), int(aggregates), ctypes.byref(h)),
               "cq_create")
        self._h = h
        self.groups = int(groups)
        self.window = int(window)
        self.last_n = 0
        if partition != PARTITION_BALANCED or workers:
            self.set_partition(partition, workers)
        if reserve:
            _check(L.cq_reserve(self._h, int(reserve)), "cq_reserve")

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            rc = lib().cq_destroy(self._h)
            self._h = None
            _check(rc, "cq_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- configuration -----------------------------------------------------
    def set_partition(self, mode: int, workers: int = 0):
        _check(lib().cq_set_partition(self._h, int(mode), int(workers)), "cq_set_partition")

    def set_key_mod(self, on: bool = True):
        """Take every key as (uint32)key mod groups (cq_set_key_mod)."""
        _check(lib().cq_set_key_mod(self._h, int(bool(on))), "cq_set_key_mod")

    def set_policy_params(self, threshold: int = 1000, pot: float = 0.5):
        _check(lib().cq_set_policy_params(self._h, int(threshold), float(pot)),
               "cq_set_policy_params")

    def policy_stats(self):
        """(moves after the last batch, max and min tuples per worker of that
        batch, moves since the technique was selected)."""
        out = (ctypes.c_int64 * 4)()
        _check(lib().cq_policy_stats(self._h, out), "cq_policy_stats")
        return tuple(int(v) for v in out)

    def reserve(self, max_batch: int):
        _check(lib().cq_reserve(self._h, int(max_batch)), "cq_reserve")

    def set_telemetry(self, flags: int):
        _check(lib().cq_set_telemetry(self._h, int(flags)), "cq_set_telemetry")

    # -- the hot path ------------------------------------------------------
    def push(self, keys, values, stream=None):
        """Enqueue one batch: ``keys``/``values`` are int32 device tensors."""
        n = keys.numel()
        if values.numel() != n:
            raise ValueError("keys and values differ in length")
        if n and (keys.dtype != values.dtype or not keys.is_cuda or not values.is_cuda
                  or not keys.is_contiguous() or not values.is_contiguous()):
            raise ValueError("keys and values must be contiguous int32 device tensors")
        _check(lib().cq_push_batch(self._h, _dptr(keys) if n else None,
                                   _dptr(values) if n else None, int(n),
                                   _stream_handle(stream)), "cq_push_batch")
        self.last_n = int(n)

    def push_results_into(self, keys, values, ids, sums, counts, avgs, n_touched, stream=None):
        """Enqueue one batch and the emission of its results into caller
        device tensors (cq_push_batch_results)."""
        n = keys.numel()
        if values.numel() != n:
            raise ValueError("keys and values differ in length")
        _check(lib().cq_push_batch_results(
            self._h, _dptr(keys) if n else None, _dptr(values) if n else None, int(n),
            _dptr(ids), _dptr(sums), _dptr(counts), _dptr(avgs), _dptr(n_touched),
            _stream_handle(stream)), "cq_push_batch_results")
        self.last_n = int(n)

    def push_results_noalloc_into(self, keys, values, ids, sums, counts, avgs, n_touched,
                                  stream=None):
        """push_results_into through the allocation-free entry point
        (cq_push_batch_results_noalloc): at most NOALLOC_MAX_BATCH tuples,
        at most NOALLOC_MAX_GROUPS groups, balanced partition."""
        n = keys.numel()
        if values.numel() != n:
            raise ValueError("keys and values differ in length")
        _check(lib().cq_push_batch_results_noalloc(
            self._h, _dptr(keys) if n else None, _dptr(values) if n else None, int(n),
            _dptr(ids), _dptr(sums), _dptr(counts), _dptr(avgs), _dptr(n_touched),
            _stream_handle(stream)), "cq_push_batch_results_noalloc")
        self.last_n = int(n)

    def push_tuples_into(self, keys, values, sums, counts, avgs, passes=0, stream=None):
        """Enqueue one batch and, per tuple, its group's window aggregate
        right after it entered (cq_push_batch_tuples): SUM / COUNT / AVG
        into caller device tensors of len(keys) entries (any may be None).
        passes = 0: incremental sums; >= 1: every window summed from
        scratch that many times."""
        n = keys.numel()
        if values.numel() != n:
            raise ValueError("keys and values differ in length")
        for t in (sums, counts, avgs):
            if t is not None and t.numel() < n:
                raise ValueError("per-tuple outputs need one entry per tuple")
        _check(lib().cq_push_batch_tuples(
            self._h, _dptr(keys) if n else None, _dptr(values) if n else None, int(n),
            int(passes), _dptr(sums), _dptr(counts), _dptr(avgs), _stream_handle(stream)),
            "cq_push_batch_tuples")
        self.last_n = int(n)

    def push_tuples(self, keys, values, passes=0, stream=None):
        """push_tuples_into with fresh device tensors; returns them."""
        import torch
        n = keys.numel()
        dev = keys.device
        sums = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        counts = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        avgs = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
        self.push_tuples_into(keys, values, sums, counts, avgs, passes, stream)
        return sums[:n], counts[:n], avgs[:n]

    def push_batches_into(self, batches, outputs, stream=None):
        """Enqueue several consecutive batches in one call, overlapped inside
        the library (cq_push_batches; up to CHAIN_BATCHES of them share one
        set of launches).  batches: list of (keys, values) device tensors
        (at most PIPE_MAX tuples each); outputs: list of (ids, sums, counts,
        avgs, n_touched) device tensors, one per batch (any of the first
        four may be None)."""
        m = len(batches)
        if len(outputs) != m:
            raise ValueError("one output tuple per batch")
        P = ctypes.c_void_p
        arrs = [(P * max(m, 1))() for _ in range(7)]
        ns = (ctypes.c_int64 * max(m, 1))()
        for i, ((k, v), out) in enumerate(zip(batches, outputs)):
            n = k.numel()
            if v.numel() != n:
                raise ValueError("keys and values differ in length")
            ns[i] = n
            arrs[0][i] = _dptr(k) if n else None
            arrs[1][i] = _dptr(v) if n else None
            for j, t in enumerate(out):
                arrs[2 + j][i] = _dptr(t) if t is not None else None
        _check(lib().cq_push_batches(self._h, m, *[ctypes.cast(a, P) for a in arrs[:2]],
                                     ctypes.cast(ns, P),
                                     *[ctypes.cast(a, P) for a in arrs[2:]],
                                     _stream_handle(stream)), "cq_push_batches")
        if m:
            self.last_n = int(ns[m - 1])

    def results_into(self, ids, sums, counts, avgs, n_touched, stream=None):
        """Enqueue the emission of the last batch's results into caller
        device tensors (any of ids/sums/counts/avgs may be None)."""
        _check(lib().cq_results(self._h, _dptr(ids), _dptr(sums), _dptr(counts), _dptr(avgs),
                                _dptr(n_touched), _stream_handle(stream)), "cq_results")

    def results(self, stream=None):
        """Host-synchronising convenience: (ids, sums, counts, avgs) as CPU
        tensors; raises CQError(ERR_KEY_RANGE) for a rejected batch."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        cap = max(1, min(self.groups, self.last_n))
        ids = torch.empty(cap, dtype=torch.int32, device=dev)
        sums = torch.empty(cap, dtype=torch.int64, device=dev)
        counts = torch.empty(cap, dtype=torch.int32, device=dev)
        avgs = torch.empty(cap, dtype=torch.float64, device=dev)
        nt = torch.empty(1, dtype=torch.int64, device=dev)
        self.results_into(ids, sums, counts, avgs, nt, stream)
        m = int(nt.cpu().item())
        if m < 0:
            raise CQError(m, "batch")
        return ids[:m].cpu(), sums[:m].cpu(), counts[:m].cpu(), avgs[:m].cpu()

    def status(self) -> int:
        return lib().cq_status(self._h)

    # -- measurement -------------------------------------------------------
    def kernel_times(self):
        """{kind: (ms, launches)} since the previous call (syncs)."""
        ms = (ctypes.c_double * len(KERNEL_KINDS))()
        ln = (ctypes.c_int64 * len(KERNEL_KINDS))()
        _check(lib().cq_kernel_times(self._h, ms, ln, len(KERNEL_KINDS)), "cq_kernel_times")
        return {k: (ms[i], ln[i]) for i, k in enumerate(KERNEL_KINDS)}

    def worker_trace(self):
        """Per-workgroup records of the last batch's per-group phase as a list
        of (hw_id, xcc_id, t_start, t_end, tuples, items) tuples."""
        cnt = ctypes.c_int64(0)
        _check(lib().cq_worker_trace(self._h, None, 0, ctypes.byref(cnt)), "cq_worker_trace")
        m = cnt.value
        buf = (ctypes.c_int64 * (6 * max(m, 1)))()
        _check(lib().cq_worker_trace(self._h, buf, m, ctypes.byref(cnt)), "cq_worker_trace")
        return [tuple(buf[6 * i:6 * i + 6]) for i in range(m)]

    def phase_trace(self, kind: int):
        """Phase clocks of the last sub-batch for kernel `kind` (0 histogram +
        plan, 1 reorder pass, 2 update): list of 8-tuples per workgroup."""
        cnt = ctypes.c_int64(0)
        _check(lib().cq_phase_trace(self._h, int(kind), None, 0, ctypes.byref(cnt)),
               "cq_phase_trace")
        m = cnt.value
        buf = (ctypes.c_int64 * (8 * max(m, 1)))()
        _check(lib().cq_phase_trace(self._h, int(kind), buf, m, ctypes.byref(cnt)),
               "cq_phase_trace")
        return [tuple(buf[8 * i:8 * i + 8]) for i in range(m)]

    def batch_plan(self):
        out = (ctypes.c_int64 * 9)()
        _check(lib().cq_batch_plan(self._h, out), "cq_batch_plan")
        keys = ("light_buckets", "heavy_groups", "light_tuples", "touched", "buckets",
                "sub_touched", "status", "tiles", "fault")
        return dict(zip(keys, list(out)))


def query_footprint(groups: int, window: int) -> int:
    """Device bytes a query allocates (cq_query_footprint); -1 if invalid."""
    return int(lib().cq_query_footprint(int(groups), int(window)))


class Server:
    """A serving loop (cq_server_*): resident queries admitted by device
    footprint, batches submitted as they arrive and run on a few streams
    while the caller keeps submitting."""

    def __init__(self, memory_budget: int = 0, lanes: int = 0, slots: int = 0):
        h = ctypes.c_void_p()
        _check(lib().cq_server_create(int(memory_budget), int(lanes), int(slots),
                                      ctypes.byref(h)), "cq_server_create")
        self._h = h
        self._keep = {}  # ticket -> tensors the request reads or writes

    def add_query(self, groups: int, window: int, aggregates: int = SUM | COUNT | AVG) -> int:
        qid = ctypes.c_int32(0)
        _check(lib().cq_server_add_query(self._h, int(groups), int(window), int(aggregates),
                                         ctypes.byref(qid)), "cq_server_add_query")
        return qid.value

    def remove_query(self, qid: int):
        _check(lib().cq_server_remove_query(self._h, int(qid)), "cq_server_remove_query")

    def submit(self, qid: int, keys, values, ids=None, sums=None, counts=None, avgs=None,
               n_touched=None) -> int:
        """Queue one batch (int32 device tensors); results go to the given
        device tensors (n_touched: int64, one entry, allocated if None).
        Returns the ticket; the tensors are kept alive until it is waited."""
        import torch
        n = keys.numel()
        if values.numel() != n:
            raise ValueError("keys and values differ in length")
        if n_touched is None:
            n_touched = torch.empty(1, dtype=torch.int64, device=keys.device)
        t = ctypes.c_int64(0)
        _check(lib().cq_server_submit(
            self._h, int(qid), _dptr(keys) if n else None, _dptr(values) if n else None, int(n),
            _dptr(ids), _dptr(sums), _dptr(counts), _dptr(avgs), _dptr(n_touched),
            ctypes.byref(t)), "cq_server_submit")
        self._keep[t.value] = (keys, values, ids, sums, counts, avgs, n_touched)
        return t.value

    def wait(self, ticket: int = -1):
        rc = lib().cq_server_wait(self._h, int(ticket))
        if ticket < 0:
            self._keep.clear()
        else:
            self._keep.pop(ticket, None)
        _check(rc, "cq_server_wait")

    def stats(self):
        out = (ctypes.c_double * 8)()
        _check(lib().cq_server_stats(self._h, out), "cq_server_stats")
        keys = ("requests", "p50_us", "p99_us", "max_us", "tuples", "tuples_per_s",
                "bytes_held", "budget")
        return dict(zip(keys, list(out)))

    def close(self):
        if getattr(self, "_h", None):
            rc = lib().cq_server_destroy(self._h)
            self._h = None
            self._keep.clear()
            _check(rc, "cq_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Multi:
    """Queries that share one input stream (cq_multi_*), spread over lanes,
    with an online autotuner.  Keeps the Query objects alive."""

    def __init__(self, queries, lanes: int = 0):
        self.queries = list(queries)
        arr = (ctypes.c_void_p * len(self.queries))(*[q._h.value for q in self.queries])
        h = ctypes.c_void_p()
        _check(lib().cq_multi_create(arr, len(self.queries), int(lanes), ctypes.byref(h)),
               "cq_multi_create")
        self._h = h

    def push(self, keys, values, stream=None):
        n = keys.numel()
        if values.numel() != n:
            raise ValueError("keys and values differ in length")
        _check(lib().cq_multi_push(self._h, _dptr(keys) if n else None,
                                   _dptr(values) if n else None, int(n),
                                   _stream_handle(stream)), "cq_multi_push")
        for q in self.queries:
            q.last_n = int(n)

    def set_graph(self, on: bool = True):
        """Replay each push as one captured HIP graph (cq_multi_set_graph)."""
        _check(lib().cq_multi_set_graph(self._h, int(bool(on))), "cq_multi_set_graph")

    def tune(self, reps: int = 2):
        _check(lib().cq_multi_tune(self._h, int(reps)), "cq_multi_tune")

    def plan(self):
        k = len(self.queries)
        modes, workers, lanes = ((ctypes.c_int32 * k)() for _ in range(3))
        ms = (ctypes.c_float * k)()
        _check(lib().cq_multi_plan(self._h, modes, workers, lanes, ms), "cq_multi_plan")
        return [{"mode": modes[i], "workers": workers[i], "lane": lanes[i], "ms": ms[i]}
                for i in range(k)]

    def close(self):
        if getattr(self, "_h", None):
            rc = lib().cq_multi_destroy(self._h)
            self._h = None
            _check(rc, "cq_multi_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass
