"""ctypes loader for the C transcription of the integer oracle (tgo_oracle.c).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the benchmark).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .model import Model, DEFAULT

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tgo_oracle.c")
# TGO_ORACLE_LIB names another build of the same source (the sanitizer test
# loads an AddressSanitizer / UBSan build this way); it is used as it is.
LIB = os.environ.get("TGO_ORACLE_LIB") or os.path.join(HERE, "libtgo_oracle.so")


class OracleSummary(ctypes.Structure):
    _fields_ = [("min_ns", ctypes.c_int64), ("max_ns", ctypes.c_int64),
                ("argmin", ctypes.c_uint64), ("argmax", ctypes.c_uint64),
                ("sum_lo", ctypes.c_uint64), ("sum_hi", ctypes.c_uint64),
                ("count", ctypes.c_uint64), ("fingerprint", ctypes.c_uint64)]


def build() -> str:
    """Compile the oracle with gcc (plain -O2, no tuning)."""
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", SRC, "-o", LIB + ".tmp"],
                   check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("TGO_ORACLE_LIB") and (
                not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        L = ctypes.CDLL(LIB)
        L.oracle_simulate.restype = ctypes.c_int64
        L.oracle_simulate.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        L.oracle_exhaustive.restype = ctypes.c_int
        L.oracle_exhaustive.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.POINTER(OracleSummary)]
        L.oracle_eval_orders.restype = ctypes.c_int
        L.oracle_eval_orders.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p]
        L.oracle_rounds_simulate.restype = ctypes.c_int64
        L.oracle_rounds_simulate.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_rounds_times.restype = ctypes.c_int
        L.oracle_rounds_times.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p]
        L.oracle_mem_simulate.restype = ctypes.c_int64
        L.oracle_mem_simulate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int]
        L.oracle_mem_times.restype = ctypes.c_int
        L.oracle_mem_times.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
        L.oracle_cke_simulate.restype = ctypes.c_int64
        L.oracle_cke_simulate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int]
        L.oracle_cke_times.restype = ctypes.c_int
        L.oracle_cke_times.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
        _lib = L
    return _lib


def _tasks(tasks) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(tasks, dtype=np.int64).reshape(-1, 3))


def simulate(tasks, order, model: Model = DEFAULT) -> int:
    t = _tasks(tasks)
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    return int(lib().oracle_simulate(t.ctypes.data, len(o), o.ctypes.data, model.q, model.p_htd,
                                     model.p_dth, model.dma_engines, None))


def eval_orders(tasks, orders, model: Model = DEFAULT) -> np.ndarray:
    t = _tasks(tasks)
    o = np.ascontiguousarray(np.asarray(orders, dtype=np.uint8))
    m, n = o.shape
    out = np.empty(m, dtype=np.int64)
    rc = lib().oracle_eval_orders(t.ctypes.data, n, model.q, model.p_htd, model.p_dth,
                                  model.dma_engines, o.ctypes.data, m, out.ctypes.data)
    assert rc == 0
    return out


def default_threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def exhaustive(tasks, model: Model = DEFAULT, lo: int = 0, hi: int | None = None, stride: int = 1,
               threads: int | None = None, per_order: bool = False):
    """Summary over ranks [lo, hi) (every stride-th rank); optional per-ordering T."""
    import math
    t = _tasks(tasks)
    n = len(t)
    if hi is None:
        hi = math.factorial(n)
    threads = threads or default_threads()
    po = np.empty(hi - lo, dtype=np.int64) if (per_order and stride == 1) else None
    s = OracleSummary()
    rc = lib().oracle_exhaustive(t.ctypes.data, n, model.q, model.p_htd, model.p_dth,
                                 model.dma_engines, lo, hi, stride, threads,
                                 po.ctypes.data if po is not None else None, ctypes.byref(s))
    assert rc == 0
    total = s.sum_lo | (s.sum_hi << 64)
    out = {"min_ns": s.min_ns, "argmin_rank": s.argmin, "max_ns": s.max_ns,
           "argmax_rank": s.argmax, "sum": total, "count": s.count,
           "mean_ns": total / s.count if s.count else float("nan"),
           "fingerprint": s.fingerprint, "threads": threads}
    if po is not None:
        out["times"] = po
    return out


def rounds_times(tasks, T: int, R: int, model: Model = DEFAULT, threads: int | None = None) -> np.ndarray:
    """NoReorder T of every ordering of T workers x R dependent tasks, by rank
    (C transcription of oracle/rounds.py)."""
    import math
    t = _tasks(tasks)
    assert len(t) == T * R
    out = np.empty(math.factorial(T) ** R, dtype=np.int64)
    rc = lib().oracle_rounds_times(t.ctypes.data, T, R, model.q, model.p_htd, model.p_dth,
                                   model.dma_engines, threads or default_threads(), out.ctypes.data)
    assert rc == 0
    return out


def mem_simulate(tasks, mem, capacity: int, order, model: Model = DEFAULT) -> int:
    """T of one ordering under the device-memory limit (C transcription of
    oracle/memory.py)."""
    t = _tasks(tasks)
    m = np.ascontiguousarray(np.asarray(mem, dtype=np.int64))
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    return int(lib().oracle_mem_simulate(t.ctypes.data, m.ctypes.data, len(t), int(capacity), o.ctypes.data,
                                         model.q, model.p_htd, model.p_dth, model.dma_engines))


def mem_times(tasks, mem, capacity: int, model: Model = DEFAULT, lo: int = 0, hi: int | None = None,
              threads: int | None = None) -> np.ndarray:
    """T under the device-memory limit for the orderings of ranks [lo, hi)."""
    import math
    t = _tasks(tasks)
    m = np.ascontiguousarray(np.asarray(mem, dtype=np.int64))
    n = len(t)
    hi = math.factorial(n) if hi is None else hi
    out = np.empty(hi - lo, dtype=np.int64)
    rc = lib().oracle_mem_times(t.ctypes.data, m.ctypes.data, n, int(capacity), model.q, model.p_htd,
                                model.p_dth, model.dma_engines, lo, hi, threads or default_threads(),
                                out.ctypes.data)
    assert rc == 0
    return out


def cke_simulate(tasks, units, capacity: int, order, model: Model = DEFAULT) -> int:
    """T of one ordering under the concurrent-kernel rule (C transcription of
    oracle/cke.py)."""
    t = _tasks(tasks)
    u = np.ascontiguousarray(np.asarray(units, dtype=np.int32))
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    return int(lib().oracle_cke_simulate(t.ctypes.data, u.ctypes.data, len(t), int(capacity), o.ctypes.data,
                                         model.q, model.p_htd, model.p_dth, model.dma_engines))


def cke_times(tasks, units, capacity: int, model: Model = DEFAULT, lo: int = 0, hi: int | None = None,
              threads: int | None = None) -> np.ndarray:
    """T under the concurrent-kernel rule for the orderings of ranks [lo, hi)."""
    import math
    t = _tasks(tasks)
    u = np.ascontiguousarray(np.asarray(units, dtype=np.int32))
    n = len(t)
    hi = math.factorial(n) if hi is None else hi
    out = np.empty(hi - lo, dtype=np.int64)
    rc = lib().oracle_cke_times(t.ctypes.data, u.ctypes.data, n, int(capacity), model.q, model.p_htd,
                                model.p_dth, model.dma_engines, lo, hi, threads or default_threads(),
                                out.ctypes.data)
    assert rc == 0
    return out
