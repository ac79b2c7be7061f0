"""The pins are discriminating: plausible mistakes planted in a private copy
of the C oracle (compiled to a temporary library, on the CPU) must each fail
at least one pin.  The real oracle is never modified."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle
import oracle_pins as P

SRC = open(oracle.SOURCE).read()

MUTANTS = {
    # the pointer to the oldest slot stops moving once the window is full,
    # so the newest value is overwritten instead of the oldest
    "evict_newest": ("    q->nextPos[g] = (q->nextPos[g] + 1) % q->W;\n",
                     "    if (q->filled[g] < q->W) q->nextPos[g] = (q->nextPos[g] + 1) % q->W;\n"),
    # COUNT reported as the window size even while the window fills
    "count_is_w": ("int32_t c = q->filled[g];", "int32_t c = q->W;"),
    # window one value short
    "window_short": ("if (q->filled[g] < q->W)\n        q->filled[g] += 1;",
                     "if (q->filled[g] < q->W - 1 || q->W == 1)\n        q->filled[g] += 1;"),
    # tuples of a batch applied in reverse arrival order
    "reverse_order": ("for (int64_t i = 0; i < n; ++i)\n        window_insert(q, keys[i], values[i]);",
                      "for (int64_t i = n - 1; i >= 0; --i)\n        window_insert(q, keys[i], values[i]);"),
    # the partial window summed from nextPos instead of from slot 0
    "partial_from_nextpos": ("s += (int64_t)win[j];",
                             "s += (int64_t)win[(q->nextPos[g] + j) % q->W];"),
    # AVG by integer division
    "avg_integer_div": ("avgs[m] = (double)s / (double)c;", "avgs[m] = (double)(s / c);"),
    # 32-bit accumulator
    "sum_int32": ("int64_t s = 0;\n    for (int32_t j", "int32_t s = 0;\n    for (int32_t j"),
    # every group emitted, touched or not
    "emit_untouched": ("if (!q->touched[g])\n            continue;\n", ""),
    # per-tuple form: the window read before the tuple enters it
    "tuple_sum_before_insert": ("window_insert(q, g, values[i]);\n        int64_t ws = window_sum(q, g);",
                                "int64_t ws = window_sum(q, g);\n        window_insert(q, g, values[i]);"),
    # per-tuple form: COUNT reported as the window size
    "tuple_count_is_w": ("int32_t wc = q->filled[g];", "int32_t wc = q->W;"),
    # per-tuple form: AVG by integer division
    "tuple_avg_integer_div": ("avgs[i] = (double)ws / (double)wc;", "avgs[i] = (double)(ws / wc);"),
}


@pytest.fixture(scope="module")
def tmpdir_mod():
    with tempfile.TemporaryDirectory() as d:
        yield d


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmpdir_mod):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    src = os.path.join(tmpdir_mod, f"{name}.c")
    lib = os.path.join(tmpdir_mod, f"lib{name}.so")
    with open(src, "w") as f:
        f.write(SRC.replace(old, new))
    hdr = os.path.join(os.path.dirname(oracle.SOURCE), "cq_oracle.h")
    with open(os.path.join(tmpdir_mod, "cq_oracle.h"), "w") as f:
        f.write(open(hdr).read())
    oracle.build(src, lib)

    # Run the pins in a child process: a mutant that corrupts memory then
    # dies there (which also counts as caught) instead of in the test runner.
    here = os.path.dirname(os.path.abspath(__file__))
    script = (
        "import sys; sys.path[:0] = [%r, %r]\n"
        "import oracle, oracle_pins as P\n"
        "make = lambda G, W: oracle.RingOracle(G, W, lib_path=%r)\n"
        "failed = []\n"
        "for pin in P.ALL_PINS:\n"
        "    try:\n"
        "        pin(make)\n"
        "    except Exception as e:\n"
        "        failed.append(pin.__name__)\n"
        "print('FAILED_PINS', failed)\n"
        "sys.exit(1 if failed else 0)\n"
    ) % (here, os.path.dirname(here), lib)
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0, f"mutant {name} passed every pin: {r.stdout[-500:]}"
