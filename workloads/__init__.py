"""Seeded synthetic stream generators (input data only).

This module produces the (key, value) int32 batches that both the CPU oracle
and the HIP path consume.  It holds none of the method's arithmetic: no
windows, no grouping, no sums.  It only draws keys and values.

Workload shapes follow the paper's experimental setting (Section 5.1): a
stream of (group id, integer attribute) tuples processed in fixed-size
batches, with keys either round-robin (the unskewed DS1), Zipf-distributed
with the id order equal to the frequency order (DS2), or Zipf with the ids
randomly permuted (DS3).  The paper does not state its Zipf exponent, so the
exponent is a parameter and the configurations below sweep it.

Seeding: every batch is drawn from its own PCG64 stream seeded with
``SeedSequence([13090634, config_id, s_index, batch_index])``; permutations
of the hot-key ranks use ``[13090634, config_id, s_index, PERM_TAG + epoch]``.
Device-side generation (``device=`` a torch CUDA device) uses torch's
Philox generator with a seed derived from the same tuple.  Host and device
streams are different arrays; whichever arrays are generated are what both
sides are given.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, Optional, Sequence, Tuple

import numpy as np

ROOT_SEED = 13090634
PERM_TAG = 1_000_000
VALUE_HI = 1_000_000          # values drawn in [0, VALUE_HI)


@dataclasses.dataclass(frozen=True)
class StreamConfig:
    """One synthetic stream: sizes and distributions (no method parameters
    beyond the window, which the query needs)."""
    name: str
    config_id: int
    groups: int
    window: int
    batch: int
    batches: int
    key_dist: str               # "uniform" | "zipf" | "roundrobin"
    zipf_s: float = 0.0
    permuted: bool = True       # DS3-like (True) or DS2-like (False)
    perm_epoch: int = 0         # redraw the hot-key permutation every this many batches (0: never)
    value_dist: str = "uniform"  # "uniform" | "normal"
    s_index: int = 0


ZIPF_SWEEP = (0.0, 0.5, 1.0, 1.5, 2.0)


def tiny() -> StreamConfig:
    """64 groups, W=1000, 100 batches of 4096 uniform keys."""
    return StreamConfig("tiny_g64_w1000", 1, 64, 1000, 4096, 100, "uniform")


def skew(s: float, permuted: bool = True, batches: int = 200) -> StreamConfig:
    """10,000 groups, W=1000, 1,048,576-tuple batches, Zipf(s) keys."""
    idx = ZIPF_SWEEP.index(s) if s in ZIPF_SWEEP else 100 + int(round(s * 100))
    name = f"skew_g10000_w1000_s{s:g}" + ("" if permuted else "_sorted")
    return StreamConfig(name, 2, 10_000, 1000, 1 << 20, batches,
                        "zipf" if s > 0 else "uniform", zipf_s=s,
                        permuted=permuted, s_index=idx + (0 if permuted else 50))


PAPER_DATASETS = ("DS1", "DS2", "DS3")


def paper_shape(dataset: str, s: float = 1.0, batches: int = 2000) -> StreamConfig:
    """The paper's own setting (Section 5.1): 40,000 groups, W=100, batches
    of 50,000 tuples (2,000 batches make its 100M-tuple stream).  DS1:
    round-robin keys; DS2: Zipf(s) with the id order equal to the frequency
    order; DS3: the same with the ids permuted.  The paper does not state its
    Zipf exponent; s is a parameter."""
    if dataset not in PAPER_DATASETS:
        raise ValueError(dataset)
    idx = PAPER_DATASETS.index(dataset) * 1000 + int(round(s * 100))
    if dataset == "DS1":
        return StreamConfig("paper_g40000_w100_ds1", 6, 40_000, 100, 50_000, batches,
                            "roundrobin", s_index=idx)
    return StreamConfig(f"paper_g40000_w100_{dataset.lower()}_s{s:g}", 6, 40_000, 100, 50_000,
                        batches, "zipf", zipf_s=s, permuted=dataset == "DS3", s_index=idx)


def drifting(batches: int = 500) -> StreamConfig:
    """2^20 groups, W=100, 16,777,216-tuple batches, Zipf s=1.2 with the hot
    permutation redrawn every 50 batches, clipped-normal values."""
    return StreamConfig("drift_g1m_w100_s1.2", 3, 1 << 20, 100, 1 << 24, batches,
                        "zipf", zipf_s=1.2, permuted=True, perm_epoch=50,
                        value_dist="normal", s_index=0)


# --------------------------------------------------------------------------
# host (numpy) generation
# --------------------------------------------------------------------------

def _rng(*words: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(words))))


def zipf_cdf(n_ranks: int, s: float) -> np.ndarray:
    """Cumulative distribution of the bounded Zipf law p_r ~ r^-s, r=1..N,
    in float64, last entry forced to exactly 1."""
    r = np.arange(1, n_ranks + 1, dtype=np.float64)
    w = r ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    return cdf


def rank_permutation(cfg: StreamConfig, epoch: int) -> np.ndarray:
    """Seeded permutation rank -> key (identity for the DS2-like order)."""
    if not cfg.permuted:
        return np.arange(cfg.groups, dtype=np.int32)
    rng = _rng(ROOT_SEED, cfg.config_id, cfg.s_index, PERM_TAG + epoch)
    return rng.permutation(cfg.groups).astype(np.int32)


def _epoch(cfg: StreamConfig, b: int) -> int:
    return b // cfg.perm_epoch if cfg.perm_epoch else 0


def host_batch(cfg: StreamConfig, b: int, n: Optional[int] = None,
               _cache: dict = {}) -> Tuple[np.ndarray, np.ndarray]:
    """Batch ``b`` of ``cfg`` as two int32 numpy arrays (keys, values)."""
    n = cfg.batch if n is None else n
    rng = _rng(ROOT_SEED, cfg.config_id, cfg.s_index, b)
    if cfg.key_dist == "roundrobin":
        t0 = b * cfg.batch
        t = np.arange(t0, t0 + n, dtype=np.int64)
        keys = (t % cfg.groups).astype(np.int32)
    elif cfg.key_dist == "uniform":
        keys = rng.integers(0, cfg.groups, n, dtype=np.int64).astype(np.int32)
    elif cfg.key_dist == "zipf":
        ck = ("cdf", cfg.groups, cfg.zipf_s)
        if ck not in _cache:
            _cache.clear()
            _cache[ck] = zipf_cdf(cfg.groups, cfg.zipf_s)
        cdf = _cache[ck]
        u = rng.random(n)
        rank = np.searchsorted(cdf, u, side="right")
        np.minimum(rank, cfg.groups - 1, out=rank)
        perm = rank_permutation(cfg, _epoch(cfg, b))
        keys = perm[rank]
    else:
        raise ValueError(cfg.key_dist)
    if cfg.key_dist == "roundrobin":
        values = (np.arange(b * cfg.batch, b * cfg.batch + n, dtype=np.int64)
                  % VALUE_HI).astype(np.int32)
    elif cfg.value_dist == "uniform":
        values = rng.integers(0, VALUE_HI, n, dtype=np.int64).astype(np.int32)
    else:
        v = np.rint(rng.normal(5e5, 1e5, n))
        values = np.clip(v, 0, VALUE_HI).astype(np.int32)
    return keys.astype(np.int32, copy=False), values


def host_batches(cfg: StreamConfig, start: int = 0,
                 count: Optional[int] = None) -> Iterator[Tuple[np.ndarray, np.ndarray]]:
    count = cfg.batches - start if count is None else count
    for b in range(start, start + count):
        yield host_batch(cfg, b)


# --------------------------------------------------------------------------
# device (torch) generation, for sizes where host generation is too slow
# --------------------------------------------------------------------------

def _torch_seed(cfg: StreamConfig, b: int) -> int:
    ss = np.random.SeedSequence([ROOT_SEED, cfg.config_id, cfg.s_index, b, 7])
    return int(ss.generate_state(1, dtype=np.uint64)[0] & ((1 << 63) - 1))


class DeviceStream:
    """Draws batches of ``cfg`` directly in device memory with torch."""

    def __init__(self, cfg: StreamConfig, device):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.gen = torch.Generator(device=self.device)
        self._cdf = None
        if cfg.key_dist == "zipf":
            self._cdf = torch.from_numpy(zipf_cdf(cfg.groups, cfg.zipf_s)).to(self.device)
        self._perm = {}

    def _perm_for(self, epoch: int):
        if epoch not in self._perm:
            self._perm.clear()
            self._perm[epoch] = self.torch.from_numpy(
                rank_permutation(self.cfg, epoch)).to(self.device)
        return self._perm[epoch]

    def batch(self, b: int, n: Optional[int] = None):
        torch = self.torch
        cfg = self.cfg
        n = cfg.batch if n is None else n
        self.gen.manual_seed(_torch_seed(cfg, b))
        if cfg.key_dist == "uniform":
            keys = torch.randint(0, cfg.groups, (n,), generator=self.gen,
                                 device=self.device, dtype=torch.int32)
        elif cfg.key_dist == "zipf":
            u = torch.rand(n, generator=self.gen, device=self.device, dtype=torch.float64)
            rank = torch.searchsorted(self._cdf, u, right=True)
            rank.clamp_(max=cfg.groups - 1)
            keys = self._perm_for(_epoch(cfg, b))[rank]
        elif cfg.key_dist == "roundrobin":
            t0 = b * cfg.batch
            keys = (torch.arange(t0, t0 + n, device=self.device, dtype=torch.int64)
                    % cfg.groups).to(torch.int32)
        else:
            raise ValueError(cfg.key_dist)
        if cfg.key_dist == "roundrobin":
            values = (torch.arange(b * cfg.batch, b * cfg.batch + n, device=self.device,
                                   dtype=torch.int64) % VALUE_HI).to(torch.int32)
        elif cfg.value_dist == "uniform":
            values = torch.randint(0, VALUE_HI, (n,), generator=self.gen,
                                   device=self.device, dtype=torch.int32)
        else:
            v = torch.randn(n, generator=self.gen, device=self.device, dtype=torch.float64)
            values = torch.clamp(torch.round(v * 1e5 + 5e5), 0, VALUE_HI).to(torch.int32)
        return keys.contiguous(), values.contiguous()


def multi_stream(batches: int = 100) -> StreamConfig:
    """The shared input of the multi-query set: 4,194,304-tuple batches of
    Zipf s=1.0 keys over [0, 2^20) with permuted hot ranks, values uniform
    in [0, 1e6).  Each query takes key mod its own group count."""
    return StreamConfig("multi_k1m_n4m_s1.0", 4, 1 << 20, 1, 1 << 22, batches, "zipf",
                        zipf_s=1.0, permuted=True, s_index=0)


def multi_queries(count: int = 64) -> list:
    """(groups, window) of the multi-query set: groups log-uniform in
    [100, 1e6], windows log-uniform in [10, 1e4] (rint(exp(U)))."""
    rng = _rng(ROOT_SEED, 4, 1)
    g = np.rint(np.exp(rng.uniform(np.log(100), np.log(1e6), count))).astype(np.int64)
    w = np.rint(np.exp(rng.uniform(np.log(10), np.log(1e4), count))).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(g, w)]


# --------------------------------------------------------------------------
# serving mix: many resident queries, batches of varying size
# --------------------------------------------------------------------------

SERVING_ID = 5


def serving_queries(count: int = 256) -> list:
    """(groups, window) of `count` resident queries: both log-uniform,
    groups in [100, 1e6] and windows in [10, 1e4] (rint(exp(U)))."""
    rng = _rng(ROOT_SEED, SERVING_ID, 1)
    g = np.rint(np.exp(rng.uniform(np.log(100), np.log(1e6), count))).astype(np.int64)
    w = np.rint(np.exp(rng.uniform(np.log(10), np.log(1e4), count))).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(g, w)]


def serving_sizes(count: int, seed: int) -> np.ndarray:
    """Batch sizes: lognormal with median 65,536 and sigma 1, clipped to
    [1,024, 4,194,304]."""
    rng = _rng(ROOT_SEED, SERVING_ID, 2, seed)
    n = np.rint(np.exp(rng.normal(np.log(65536), 1.0, count)))
    return np.clip(n, 1024, 1 << 22).astype(np.int64)


class ServingBatches:
    """Device batches of query q (groups G): Zipf s=1.5 keys over G ranks
    whose hot set (the rank -> id permutation) is redrawn per epoch, values
    uniform in [0, 1e6)."""

    def __init__(self, device, zipf_s: float = 1.5):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.s = zipf_s
        self.gen = torch.Generator(device=self.device)

    def batch(self, q: int, groups: int, epoch: int, i: int, n: int):
        torch = self.torch
        ss = np.random.SeedSequence([ROOT_SEED, SERVING_ID, 3, q, epoch, i])
        self.gen.manual_seed(int(ss.generate_state(1, dtype=np.uint64)[0] & ((1 << 63) - 1)))
        r = torch.arange(1, groups + 1, device=self.device, dtype=torch.float64)
        cdf = torch.cumsum(r.pow(-self.s), 0)
        cdf /= cdf[-1].clone()
        u = torch.rand(n, generator=self.gen, device=self.device, dtype=torch.float64)
        rank = torch.searchsorted(cdf, u, right=True).clamp_(max=groups - 1)
        pss = np.random.SeedSequence([ROOT_SEED, SERVING_ID, 4, q, epoch])
        self.gen.manual_seed(int(pss.generate_state(1, dtype=np.uint64)[0] & ((1 << 63) - 1)))
        perm = torch.randperm(groups, generator=self.gen, device=self.device).to(torch.int32)
        keys = perm[rank].contiguous()
        values = torch.randint(0, VALUE_HI, (n,), generator=self.gen, device=self.device,
                               dtype=torch.int32)
        return keys, values


def probe_batch(groups: int) -> Tuple[np.ndarray, np.ndarray]:
    """One (g, 0) tuple for every group g, in ascending g."""
    return np.arange(groups, dtype=np.int32), np.zeros(groups, dtype=np.int32)


def reinterleave(keys: np.ndarray, values: np.ndarray, seed: int
                 ) -> Tuple[np.ndarray, np.ndarray]:
    """A random re-interleaving of the tuples that keeps every key's own
    subsequence in its original order (a random merge of per-key lists)."""
    rng = _rng(ROOT_SEED, 99, seed)
    n = len(keys)
    # Assign every tuple a random slot, then order slots of one key so that
    # its tuples keep their original relative order.
    slots = rng.permutation(n)
    order_by_key = np.argsort(keys, kind="stable")
    slots_sorted_per_key = np.empty(n, dtype=np.int64)
    ks = keys[order_by_key]
    bounds = np.flatnonzero(np.diff(ks)) + 1
    starts = np.concatenate(([0], bounds))
    ends = np.concatenate((bounds, [n]))
    sl = slots[order_by_key]
    for a, e in zip(starts, ends):
        slots_sorted_per_key[a:e] = np.sort(sl[a:e])
    new_pos = np.empty(n, dtype=np.int64)
    new_pos[order_by_key] = slots_sorted_per_key
    out_k = np.empty_like(keys)
    out_v = np.empty_like(values)
    out_k[new_pos] = keys
    out_v[new_pos] = values
    return out_k, out_v
