"""The oracle's output on the tiny configuration matches the digest that
tests/golden/make_golden.py stored (written by calling only the oracle)."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402


def test_tiny_oracle_digest_unchanged():
    want = open(os.path.join(HERE, "golden", "tiny_oracle_digest.txt")).read().strip()
    assert make_golden.digest() == want
