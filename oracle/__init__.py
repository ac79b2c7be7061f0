"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Python access to the plain C ring-buffer oracle (``cq_oracle.c``) and to the
pure-Python brute force (``brute.py``).  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import this package; the GPU
library never does, and this package imports nothing from it.

What it computes is the continuous sliding-window group-by of the paper
(Section 3 problem statement, Section 3.2 window store with nextPos,
Section 5.1 from-scratch window sum); see ``cq_oracle.h`` for the readings
taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "cq_oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")

ERR_INVALID = -1
ERR_OOM = -2
ERR_KEY_RANGE = -3


def build(source: str = SOURCE, output: str = LIBRARY, defines: Tuple[str, ...] = ()) -> str:
    """Compile the C oracle with gcc into a shared library."""
    cmd = ["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           *[f"-D{d}" for d in defines], "-I", _HERE, source, "-o", output, "-lpthread"]
    subprocess.run(cmd, check=True)
    return output


def _load(path: str) -> ctypes.CDLL:
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_create.argtypes = [i64, ctypes.c_int32, ctypes.POINTER(P)]
    lib.oracle_create.restype = ctypes.c_int
    lib.oracle_destroy.argtypes = [P]
    lib.oracle_destroy.restype = None
    lib.oracle_push.argtypes = [P, P, P, i64, P, P, P, P, P]
    lib.oracle_push.restype = ctypes.c_int
    lib.oracle_push_mt.argtypes = [P, P, P, i64, P, P, P, P, P, ctypes.c_int]
    lib.oracle_push_mt.restype = ctypes.c_int
    lib.oracle_push_tuples.argtypes = [P, P, P, i64, P, P, P]
    lib.oracle_push_tuples.restype = ctypes.c_int
    lib.oracle_window.argtypes = [P, i64, P]
    lib.oracle_window.restype = ctypes.c_int32
    return lib


_LIBS: dict = {}


def library(path: Optional[str] = None) -> ctypes.CDLL:
    path = path or LIBRARY
    if path not in _LIBS:
        if path == LIBRARY and (not os.path.exists(LIBRARY)
                                or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE)):
            build()
        _LIBS[path] = _load(path)
    return _LIBS[path]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


class RingOracle:
    """One continuous query evaluated on the CPU by the C oracle."""

    def __init__(self, groups: int, window: int, threads: int = 1,
                 lib_path: Optional[str] = None):
        self.lib = library(lib_path)
        self.groups = int(groups)
        self.window = int(window)
        self.threads = int(threads)
        h = ctypes.c_void_p()
        rc = self.lib.oracle_create(self.groups, self.window, ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.oracle_destroy(self._h)
            self._h = None

    __del__ = close

    def push(self, keys: np.ndarray, values: np.ndarray):
        """Apply a batch; returns (ids, sums, counts, avgs) numpy arrays.
        Raises OracleError(-3) if a key is out of range (state unchanged)."""
        keys = np.ascontiguousarray(keys, dtype=np.int32)
        values = np.ascontiguousarray(values, dtype=np.int32)
        n = len(keys)
        assert len(values) == n
        # room for every group: a touched set never exceeds min(groups, n),
        # and the extra room keeps a faulty emitter from writing out of bounds
        cap = max(1, self.groups)
        ids = np.empty(cap, np.int32)
        sums = np.empty(cap, np.int64)
        counts = np.empty(cap, np.int32)
        avgs = np.empty(cap, np.float64)
        nt = ctypes.c_int64(0)
        args = (self._h, _ptr(keys), _ptr(values), n, _ptr(ids), _ptr(sums),
                _ptr(counts), _ptr(avgs), ctypes.byref(nt))
        if self.threads > 1:
            rc = self.lib.oracle_push_mt(*args, self.threads)
        else:
            rc = self.lib.oracle_push(*args)
        if rc != 0:
            raise OracleError(rc)
        m = nt.value
        return ids[:m], sums[:m], counts[:m], avgs[:m]

    def push_tuples(self, keys: np.ndarray, values: np.ndarray):
        """Apply a batch tuple by tuple; returns (sums, counts, avgs), one
        entry per tuple: its group's window right after that tuple entered
        (Section 5.1's per-tuple, from-scratch aggregate)."""
        keys = np.ascontiguousarray(keys, dtype=np.int32)
        values = np.ascontiguousarray(values, dtype=np.int32)
        n = len(keys)
        assert len(values) == n
        sums = np.empty(max(n, 1), np.int64)
        counts = np.empty(max(n, 1), np.int32)
        avgs = np.empty(max(n, 1), np.float64)
        rc = self.lib.oracle_push_tuples(self._h, _ptr(keys), _ptr(values), n, _ptr(sums),
                                         _ptr(counts), _ptr(avgs))
        if rc != 0:
            raise OracleError(rc)
        return sums[:n], counts[:n], avgs[:n]

    def window_of(self, group: int) -> np.ndarray:
        out = np.empty(self.window, np.int32)
        f = self.lib.oracle_window(self._h, int(group), _ptr(out))
        return out[:f]
