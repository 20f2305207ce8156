"""Runs every routine of the C oracle on small random inputs and checks each
against the Python oracle.  Meant to run in a child process whose C oracle is
a sanitizer build (see tests/test_sanitizers.py); prints one line per routine."""
import itertools
import math
import sys

import numpy as np

from oracle import cke, cmodel, memory, rounds
from oracle import model as M

print("oracle library", cmodel.LIB, flush=True)
rng = np.random.default_rng(71)
models = [M.DEFAULT, M.PAPER_EXAMPLE, M.Model(4, 3, 3, 1), M.Model(2, 1, 1, 2)]


def tasks_of(n, hi=3_000_000):
    return rng.integers(0, hi, size=(n, 3)).astype(np.int64)


# simulate and eval_orders, every N up to 16
for n in range(1, 17):
    t = tasks_of(n)
    for m in models:
        orders = np.array([rng.permutation(n) for _ in range(4)], dtype=np.uint8)
        got = cmodel.eval_orders(t, orders, m)
        for o, g in zip(orders, got):
            assert g == M.simulate(t, list(o), m) == cmodel.simulate(t, list(o), m)
print("simulate/eval_orders ok", flush=True)

# exhaustive with several threads, per-ordering output and a stride
for n in (1, 2, 5, 7):
    t = tasks_of(n)
    for m in models[:2]:
        ref = M.exhaustive(t, m)
        got = cmodel.exhaustive(t, m, threads=3, per_order=True)
        for k in ("min_ns", "max_ns", "argmin_rank", "argmax_rank", "sum", "count"):
            assert got[k] == ref[k], (n, k)
        assert list(got["times"]) == M.all_times(t, m)
        part = cmodel.exhaustive(t, m, lo=1, hi=math.factorial(n), stride=2, threads=2)
        assert part["count"] == (math.factorial(n) - 1 + 1) // 2
print("exhaustive ok", flush=True)

# rounds (T workers x R dependent tasks)
for T, R in ((2, 2), (3, 2), (2, 3)):
    t = tasks_of(T * R)
    for m in models[:2]:
        got = cmodel.rounds_times(t, T, R, m, threads=2)
        ref = rounds.noreorder_times(t, T, R, m)
        assert list(got) == list(ref)
print("rounds ok", flush=True)

# memory-limited groups
for n in (3, 6):
    t = tasks_of(n)
    mem = rng.integers(1, 100, size=n).astype(np.int64)
    for cap in (int(mem.max()), int(mem.sum())):
        for m in models[:2]:
            got = cmodel.mem_times(t, mem, cap, m, threads=2)
            ref = memory.all_times(t, mem, cap, m)
            assert list(got) == list(ref)
            o = list(rng.permutation(n))
            assert cmodel.mem_simulate(t, mem, cap, o, m) == memory.simulate(t, mem, cap, o, m)
print("memory ok", flush=True)

# concurrent kernels
for n in (3, 6):
    t = tasks_of(n)
    for cap in (1, 2, 4):
        units = rng.integers(1, cap + 1, size=n).astype(np.int32)
        for m in models[:2]:
            got = cmodel.cke_times(t, units, cap, m, threads=2)
            ref = cke.all_times(t, units, cap, m)
            assert list(got) == list(ref)
            o = list(rng.permutation(n))
            assert cmodel.cke_simulate(t, units, cap, o, m) == cke.simulate(t, units, cap, o, m)
print("cke ok", flush=True)
print("workout done", flush=True)
sys.exit(0)
