"""The CPU oracle against its pins (see oracle_pins.py for what each rests on)."""
import numpy as np
import pytest

import oracle_pins as P
from oracle import RingOracle
from oracle.brute import BruteForce
from workloads import host_batch, tiny


def _single(G, W):
    return RingOracle(G, W)


def _multi(G, W):
    return RingOracle(G, W, threads=4)


@pytest.mark.parametrize("make", [_single, _multi], ids=["1thread", "4threads"])
@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin, make):
    pin(make)


def test_bruteforce_itself_on_hand_example():
    """A worked example by hand, W=3, two groups:
    batch 1: (0,1) (1,10) (0,2) (0,3) (0,4)  -> group 0 window [2,3,4] = 9,
             group 1 window [10] = 10;
    batch 2: (1,20) (1,30) (1,40) (0,5)      -> group 0 [3,4,5] = 12,
             group 1 [20,30,40] = 90 (10 evicted)."""
    bf = BruteForce(2, 3)
    assert bf.push([0, 1, 0, 0, 0], [1, 10, 2, 3, 4]) == [(0, 9, 3, 3.0), (1, 10, 1, 10.0)]
    assert bf.push([1, 1, 1, 0], [20, 30, 40, 5]) == [(0, 12, 3, 4.0), (1, 90, 3, 30.0)]
    ora = RingOracle(2, 3)
    ids, sums, counts, avgs = ora.push(np.array([0, 1, 0, 0, 0], np.int32),
                                       np.array([1, 10, 2, 3, 4], np.int32))
    assert ids.tolist() == [0, 1] and sums.tolist() == [9, 10] and counts.tolist() == [3, 1]
    assert ora.window_of(0).tolist() == [2, 3, 4]
    ids, sums, counts, avgs = ora.push(np.array([1, 1, 1, 0], np.int32),
                                       np.array([20, 30, 40, 5], np.int32))
    assert sums.tolist() == [12, 90] and avgs.tolist() == [4.0, 30.0]
    assert ora.window_of(1).tolist() == [20, 30, 40]


def test_multithread_equals_single_on_tiny_config():
    cfg = tiny()
    a = RingOracle(cfg.groups, cfg.window)
    b = RingOracle(cfg.groups, cfg.window, threads=8)
    for bi in range(30):
        k, v = host_batch(cfg, bi)
        ra, rb = a.push(k, v), b.push(k, v)
        for x, y in zip(ra, rb):
            assert np.array_equal(x, y)


def test_oracle_rejects_bad_arguments():
    from oracle import OracleError
    with pytest.raises(OracleError):
        RingOracle(0, 5)
    with pytest.raises(OracleError):
        RingOracle(5, 0)
