"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad host-side arguments before touching the device (CPU only)."""
import ctypes
import re

import pytest

import paper_1309_0634_amd as cq


def _declared_functions():
    src = open(cq.HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(cq_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    try:
        return cq.lib()
    except ImportError:
        import __graft_entry__
        __graft_entry__.build()
        return cq.lib()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("cq_create", "cq_push_batch", "cq_results", "cq_destroy", "cq_strerror"):
        assert required in names


def test_every_declared_symbol_is_exported(L):
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_strerror(L):
    assert cq.strerror(cq.OK) == "success"
    assert "key" in cq.strerror(cq.ERR_KEY_RANGE)
    assert cq.strerror(12345) == "unknown status code"


def test_create_rejects_bad_arguments_without_device(L):
    h = ctypes.c_void_p()
    for groups, window, aggs in [(0, 10, 7), (-5, 10, 7), (10, 0, 7), (10, -1, 7),
                                 (10, cq.MAX_WINDOW + 1, 7), (10, 10, 0), (10, 10, 8),
                                 (1 << 31, 10, 7)]:
        assert L.cq_create(groups, window, aggs, ctypes.byref(h)) == cq.ERR_INVALID
        assert h.value is None
    assert L.cq_create(10, 10, 7, None) == cq.ERR_INVALID


def test_null_handles_are_rejected(L):
    assert L.cq_push_batch(None, None, None, 0, None) == cq.ERR_INVALID
    assert L.cq_results(None, None, None, None, None, None, None) == cq.ERR_INVALID
    assert L.cq_set_partition(None, 0, 0) == cq.ERR_INVALID
    assert L.cq_reserve(None, 10) == cq.ERR_INVALID
    assert L.cq_status(None) == cq.ERR_INVALID
    assert L.cq_set_telemetry(None, 1) == cq.ERR_INVALID
    assert L.cq_batch_plan(None, None) == cq.ERR_INVALID
    assert L.cq_push_batches(None, 1, None, None, None, None, None, None, None, None,
                             None) == cq.ERR_INVALID
    assert L.cq_push_batch_tuples(None, None, None, 0, 0, None, None, None,
                                  None) == cq.ERR_INVALID
    assert L.cq_set_policy_params(None, 1000, 0.5) == cq.ERR_INVALID
    assert L.cq_policy_stats(None, None) == cq.ERR_INVALID
    assert L.cq_server_add_query(None, 10, 10, 7, None) == cq.ERR_INVALID
    assert L.cq_server_remove_query(None, 0) == cq.ERR_INVALID
    assert L.cq_server_submit(None, 0, None, None, 0, None, None, None, None, None,
                              None) == cq.ERR_INVALID
    assert L.cq_server_wait(None, -1) == cq.ERR_INVALID
    assert L.cq_server_stats(None, None) == cq.ERR_INVALID
    assert L.cq_server_create(-1, 0, 0, None) == cq.ERR_INVALID
    assert L.cq_server_destroy(None) == cq.OK
    assert L.cq_set_key_mod(None, 1) == cq.ERR_INVALID
    assert L.cq_query_groups(None, None) == cq.ERR_INVALID
    assert L.cq_multi_create(None, 1, 0, None) == cq.ERR_INVALID
    assert L.cq_multi_push(None, None, None, 0, None) == cq.ERR_INVALID
    assert L.cq_multi_tune(None, 2) == cq.ERR_INVALID
    assert L.cq_multi_plan(None, None, None, None, None) == cq.ERR_INVALID
    assert L.cq_multi_set_graph(None, 1) == cq.ERR_INVALID
    assert L.cq_multi_destroy(None) == cq.OK
    assert L.cq_destroy(None) == cq.OK


def test_binding_names_match_header():
    for name in ("cq_create", "cq_reserve", "cq_set_partition", "cq_push_batch", "cq_results",
                 "cq_status", "cq_destroy", "cq_strerror", "cq_set_telemetry",
                 "cq_kernel_times", "cq_worker_trace", "cq_batch_plan", "cq_phase_trace",
                 "cq_push_batches", "cq_push_batch_results", "cq_push_batch_tuples",
                 "cq_set_policy_params", "cq_policy_stats", "cq_policy_apply"):
        assert name in _declared_functions()


def test_header_constants_match_binding():
    src = open(cq.HEADER).read()

    def val(name):
        m = re.search(r"#define\s+%s\s+\(?(-?\w+)" % name, src)
        return int(m.group(1).rstrip("u"), 0)

    assert val("CQ_SUM") == cq.SUM and val("CQ_COUNT") == cq.COUNT and val("CQ_AVG") == cq.AVG
    assert val("CQ_ERR_KEY_RANGE") == cq.ERR_KEY_RANGE
    assert val("CQ_PARTITION_STATIC") == cq.PARTITION_STATIC
    assert val("CQ_PIPE_MAX") == cq.PIPE_MAX
    assert val("CQ_CHAIN_BATCHES") == cq.CHAIN_BATCHES
    assert val("CQ_KERNEL_KINDS") == len(cq.KERNEL_KINDS)
    assert val("CQ_KERNEL_TUPLES") == cq.KERNEL_KINDS.index("tuples")
    assert val("CQ_TUPLE_MAX_WINDOW") == cq.TUPLE_MAX_WINDOW
    assert val("CQ_TUPLE_MAX_PASSES") == cq.TUPLE_MAX_PASSES
    assert val("CQ_TUPLE_MAX_GROUPS") == cq.TUPLE_MAX_GROUPS
    for name, v in cq.POLICIES.items():
        assert val("CQ_PARTITION_" + name.upper()) == v


def test_query_footprint(L):
    """The admission size: the window store dominates and grows with G*W;
    invalid sizes give -1 (host arithmetic only)."""
    f = cq.query_footprint
    assert f(0, 10) == -1 and f(10, 0) == -1 and f(10, cq.MAX_WINDOW + 1) == -1
    base = f(10_000, 1)
    assert f(10_000, 1000) - base >= 4 * 10_000 * 999
    assert f(10_000, 1000) - base <= 4 * 10_000 * 999 + 2 * 4096
    assert f(1_000_000, 100) > f(100_000, 100) > f(10_000, 100)
    assert all(f(g, w) % 4096 == 0 for g, w in [(1, 1), (777, 13), (123_457, 99)])


def test_division_free_remainder():
    """The kernels reduce a key mod G without dividing: with
    M = floor((2^64-1)/G) + 1 (M = 1 for G = 1), (uint32)a mod G is the high
    64 bits of (M*a mod 2^64)*G.  Checked here against % (the identity the
    device code relies on), at the edges and on random 32-bit values."""
    import random
    m64 = (1 << 64) - 1
    rnd = random.Random(5)
    for G in [1, 2, 3, 7, 100, 9999, 10000, 16384, 65537, 1 << 20, 1_000_000,
              (1 << 31) - 2, (1 << 31) - 1]:
        M = 1 if G == 1 else m64 // G + 1
        for a in [0, 1, G - 1, G, 2 * G - 1, (1 << 31) - 1, 1 << 31, (1 << 32) - 1] + \
                [rnd.getrandbits(32) for _ in range(3000)]:
            a &= (1 << 32) - 1
            assert ((((M * a) & m64) * G) >> 64) == a % G, (a, G)

def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asking for more exits with a message
    before anything touches a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
