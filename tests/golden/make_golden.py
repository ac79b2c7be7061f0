"""Writes tests/golden/tiny_oracle_digest.txt: a SHA-256 digest of the CPU
oracle's full output on the tiny configuration (64 groups, W=1000, 100
batches of 4096 uniform keys).  It calls only the oracle and the input
generators.  The paper prints no worked example to store instead, so this
file only guards the oracle against unintended changes; what makes the
oracle right is the pin suite (tests/oracle_pins.py)."""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import RingOracle  # noqa: E402
from workloads import host_batches, tiny  # noqa: E402


def digest() -> str:
    cfg = tiny()
    ora = RingOracle(cfg.groups, cfg.window)
    h = hashlib.sha256()
    for keys, values in host_batches(cfg):
        for arr in ora.push(keys, values):
            h.update(arr.tobytes())
    return h.hexdigest()


if __name__ == "__main__":
    with open(os.path.join(HERE, "tiny_oracle_digest.txt"), "w") as f:
        f.write(digest() + "\n")
