"""ctypes front end of the CPU oracle (``pdd_oracle.c``).

Test infrastructure only: the test suite, the smoke check and the
benchmark's CPU-baseline leg call it; the product path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdd_oracle.c")
LIB = os.path.join(HERE, "_build", "libpdd_oracle.so")

_lib = None

ERRORS = {
    -1: "invalid argument", -2: "out of memory",
    -10: "a re-cost increased a cost", -11: "removal keys did not strictly decrease",
    -12: "kept count differs from keep", -13: "maintained cost differs from a fresh one",
    -14: "a kept key ranks above the last removed key",
}


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/_build``."""
    if not force and os.path.exists(LIB):
        return LIB
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", tmp],
                   check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.pddo_term.restype = ctypes.c_uint64
        lib.pddo_term.argtypes = [i64]
        lib.pddo_knn.restype = ctypes.c_int
        lib.pddo_knn.argtypes = [P, i64, i32, P, P]
        lib.pddo_knn_cost.restype = ctypes.c_int
        lib.pddo_knn_cost.argtypes = [P, i64, i32, i32, P, P, P]
        lib.pddo_decimate.restype = ctypes.c_int
        lib.pddo_decimate.argtypes = [P, i64, i32, i32, i64, P, P, P, i32, P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _pts(xyz):
    a = np.ascontiguousarray(xyz, dtype=np.int32)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("xyz must be [n, 3]")
    return a


def _check(rc):
    if rc != 0:
        raise OracleError(ERRORS.get(rc, "error %d" % rc))


def term(d2: int) -> int:
    return int(_load().pddo_term(int(d2)))


def knn(xyz, K: int):
    """(nbr [n, K] int32, d2 [n, K] int64) sorted by (d2, index), -1 padded."""
    P = _pts(xyz)
    n = P.shape[0]
    nbr = np.empty((n, K), dtype=np.int32)
    d2 = np.empty((n, K), dtype=np.int64)
    _check(_load().pddo_knn(_ptr(P), n, K, _ptr(nbr), _ptr(d2)))
    return nbr, d2


def knn_cost(xyz, k: int, b: int = 0):
    """(nbr [n, k+b] int32, r2k [n] int64, cost [n] uint64) of the full cloud."""
    P = _pts(xyz)
    n = P.shape[0]
    nbr = np.empty((n, k + b), dtype=np.int32)
    r2k = np.empty(n, dtype=np.int64)
    cost = np.empty(n, dtype=np.uint64)
    _check(_load().pddo_knn_cost(_ptr(P), n, k, b, _ptr(nbr), _ptr(r2k), _ptr(cost)))
    return nbr, r2k, cost


def decimate(xyz, k: int, keep: int, b: int = 6, check: bool = False, stats: bool = False):
    """Greedy decimation: (kept [keep] ascending, order [n-keep], order_cost [n-keep])."""
    P = _pts(xyz)
    n = P.shape[0]
    kept = np.empty(keep, dtype=np.int32)
    order = np.empty(n - keep, dtype=np.int32)
    order_cost = np.empty(n - keep, dtype=np.uint64)
    st = np.zeros(4, dtype=np.int64)
    _check(_load().pddo_decimate(_ptr(P), n, k, b, keep, _ptr(kept), _ptr(order), _ptr(order_cost),
                                 1 if check else 0, _ptr(st)))
    if stats:
        return kept, order, order_cost, st
    return kept, order, order_cost
