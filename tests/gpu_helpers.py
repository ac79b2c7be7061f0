"""Shared helpers of the GPU parity tests: run a stream through the HIP path
(through the C ABI) and through the CPU oracle, and compare bit for bit."""
from __future__ import annotations

import sys

import numpy as np

import paper_1309_0634_amd as cq
from oracle import RingOracle


def device():
    import torch
    return torch.device("cuda", 0)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device())


def note(msg: str):
    """Name the case on stdout (flushed) before its GPU work starts."""
    print(msg, flush=True)
    sys.stdout.flush()


def assert_same(got, want, ctx: str):
    """got: (ids, sums, counts, avgs) torch CPU tensors; want: numpy arrays."""
    names = ("ids", "sums", "counts", "avgs")
    g_ids = got[0].numpy()
    assert len(g_ids) == len(want[0]), f"{ctx}: {len(g_ids)} touched vs oracle {len(want[0])}"
    for g, w, name in zip(got, want, names):
        g = g.numpy()
        if g.dtype == np.float64:
            same = np.array_equal(g.view(np.int64), np.asarray(w, np.float64).view(np.int64))
        else:
            same = np.array_equal(g, w)
        if not same:
            bad = np.flatnonzero(g != w) if g.dtype != np.float64 else \
                np.flatnonzero(g.view(np.int64) != np.asarray(w, np.float64).view(np.int64))
            i = int(bad[0])
            raise AssertionError(f"{ctx}: {name} differs at {len(bad)} entries; first at {i}: "
                                 f"gpu {g[i]!r} oracle {w[i]!r} (group {want[0][i]})")


class Pair:
    """A GPU query and a CPU oracle fed the same batches."""

    def __init__(self, groups, window, partition=cq.PARTITION_BALANCED, workers=0,
                 oracle_threads=1):
        self.q = cq.Query(groups, window, partition=partition, workers=workers)
        self.o = RingOracle(groups, window, threads=oracle_threads)

    def step(self, keys, values, ctx="", dkeys=None, dvalues=None):
        if dkeys is None:
            dkeys, dvalues = to_dev(keys), to_dev(values)
        self.q.push(dkeys, dvalues)
        got = self.q.results()
        want = self.o.push(keys, values)
        assert_same(got, want, ctx)
        return got

    def close(self):
        self.q.close()
        self.o.close()
