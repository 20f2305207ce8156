"""Seeded synthetic task-group generators.

This module only draws inputs.  It holds none of the model's arithmetic, so
both the GPU path and the CPU oracle can be fed from it.

A task is the triple (HtD, K, DtH) of solo durations in integer nanoseconds
(Section 3 and Section 4.1: every task is an HtD transfer, a kernel and a DtH
transfer executed in that order).  The paper's own synthetic tasks (Table of
synthetic tasks, Section 4.3) are fractions of a 10 ms unit; its real tasks
(Table of command-time ranges, Section 6.1) span roughly 0.01-15 ms per command
and are classed dominant-kernel (DK: HtD + DtH <= K) or dominant-transfer (DT).
The generators below stand in for those workloads with log-uniform draws.

Draw convention: numpy ``Generator(PCG64(seed))``; tasks row-major, fields in
the order (h, k, d); a duration with range [lo, hi] is
``rint(exp(ln lo + u * (ln hi - ln lo)))`` for ``u = rng.random()``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

US = 1_000
MS = 1_000_000

# dominant-kernel / dominant-transfer ranges (ns): the long stage draws from
# [1 ms, 20 ms], the short stages from [0.1 ms, 2 ms].
LONG = (1 * MS, 20 * MS)
SHORT = (100 * US, 2 * MS)


def _logu(rng: np.random.Generator, lo: int, hi: int) -> int:
    u = rng.random()
    return int(np.rint(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))


def _task(rng: np.random.Generator, dominant_kernel: bool) -> tuple[int, int, int]:
    if dominant_kernel:
        rh, rk, rd = SHORT, LONG, SHORT
    else:
        rh, rk, rd = LONG, SHORT, LONG
    h = _logu(rng, *rh)
    k = _logu(rng, *rk)
    d = _logu(rng, *rd)
    return h, k, d


def single_group_uniform(n: int = 8, seed: int = 0, lo: int = 10 * US, hi: int = 10 * MS) -> np.ndarray:
    """Every field log-uniform in [lo, hi] ns.  Default: N=8, [10 us, 10 ms], seed 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n, 3), dtype=np.int64)
    for i in range(n):
        for f in range(3):
            out[i, f] = _logu(rng, lo, hi)
    return out


def single_group_mixed(n: int = 12, seed: int = 1) -> np.ndarray:
    """First n/2 tasks dominant-kernel, the rest dominant-transfer.  Default N=12, seed 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n, 3), dtype=np.int64)
    for i in range(n):
        out[i] = _task(rng, i < n // 2)
    return out


@dataclass
class Batch:
    """Groups in CSR form: tasks[offs[g]:offs[g+1]] is group g."""

    tasks: np.ndarray  # int64 [T, 3]
    offs: np.ndarray  # int32 [G + 1]
    labels: np.ndarray  # int8 [G] (group label) or [T] (task label); 1 = DK

    @property
    def n_groups(self) -> int:
        return len(self.offs) - 1

    def sizes(self) -> np.ndarray:
        return np.diff(self.offs)

    def group(self, g: int) -> np.ndarray:
        return self.tasks[self.offs[g]:self.offs[g + 1]]


def batch_groups(n_groups: int = 4096, n_lo: int = 4, n_hi: int = 10, seed: int = 2,
                 per_task_label: bool = False) -> Batch:
    """Groups of uneven size N ~ U{n_lo..n_hi}.

    Per group, in draw order: N, then (group label, if per_task_label is False),
    then the tasks (each preceded by its own label draw if per_task_label).
    A label is DK with probability 0.5.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    rows, offs, labels = [], [0], []
    for _ in range(n_groups):
        n = int(rng.integers(n_lo, n_hi + 1))
        if not per_task_label:
            dk = bool(rng.random() < 0.5)
            labels.append(int(dk))
        for _ in range(n):
            if per_task_label:
                dk = bool(rng.random() < 0.5)
                labels.append(int(dk))
            rows.append(_task(rng, dk))
        offs.append(offs[-1] + n)
    return Batch(np.asarray(rows, dtype=np.int64).reshape(-1, 3),
                 np.asarray(offs, dtype=np.int32), np.asarray(labels, dtype=np.int8))


def fixed_size_groups(n_groups: int, n: int, seed: int) -> Batch:
    """n_groups groups of exactly n tasks, labels drawn per task (mixed groups)."""
    return batch_groups(n_groups, n, n, seed, per_task_label=True)


@dataclass
class Arrivals:
    """A Poisson request stream: arrival times (ns) and one group per request."""

    t_ns: np.ndarray  # int64 [R]
    batch: Batch


def poisson_arrivals(rate_per_s: float = 20_000.0, duration_s: float = 1.0, n_lo: int = 4,
                     n_hi: int = 16, seed: int = 4) -> Arrivals:
    """Exponential gaps with mean 1/rate; every request carries a group with
    N ~ U{n_lo..n_hi} and per-task DK/DT labels (p = 0.5)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_req = int(rate_per_s * duration_s)
    gaps = rng.exponential(1e9 / rate_per_s, size=n_req)
    t = np.cumsum(gaps).astype(np.int64)
    b = batch_groups(n_req, n_lo, n_hi, seed + 1_000_000, per_task_label=True)
    return Arrivals(t, b)


def poisson_stream(rate_per_s: float, duration_s: float, pool: Batch, seed: int) -> Arrivals:
    """Exponential gaps with mean 1/rate; request i carries pool group idx[i],
    idx uniform over the pool (with replacement).  The gaps are drawn first,
    then the indices, from one PCG64(seed) stream.  Drawing from a fixed pool
    keeps high-rate streams cheap to build."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_req = int(rate_per_s * duration_s)
    gaps = rng.exponential(1e9 / rate_per_s, size=n_req)
    t = np.cumsum(gaps).astype(np.int64)
    idx = rng.integers(0, pool.n_groups, size=n_req)
    sizes = pool.sizes()[idx].astype(np.int64)
    offs = np.zeros(n_req + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    rows = np.repeat(pool.offs[:-1][idx].astype(np.int64) - offs[:-1], sizes) + np.arange(offs[-1])
    labels = pool.labels[rows] if len(pool.labels) == len(pool.tasks) else pool.labels[idx]
    return Arrivals(t, Batch(pool.tasks[rows], offs.astype(np.int32), labels))


# The paper's synthetic tasks T0..T7 in fractions of the 10 ms unit (Table of
# synthetic tasks), and the five 4-task benchmarks BK0..BK100 (Table of
# synthetic benchmarks).
PAPER_TASKS_UNITS = {
    "T0": (0.1, 0.8, 0.1), "T1": (0.2, 0.7, 0.1), "T2": (0.3, 0.6, 0.1), "T3": (0.1, 0.7, 0.2),
    "T4": (0.6, 0.2, 0.2), "T5": (0.2, 0.2, 0.6), "T6": (0.4, 0.2, 0.4), "T7": (0.8, 0.1, 0.1),
}
PAPER_BENCHMARKS = {
    "BK0": ("T6", "T7", "T4", "T5"),
    "BK25": ("T0", "T4", "T6", "T7"),
    "BK50": ("T0", "T1", "T4", "T5"),
    "BK75": ("T0", "T1", "T2", "T4"),
    "BK100": ("T0", "T1", "T2", "T3"),
}
PAPER_UNIT_NS = 10 * MS


def paper_benchmark(name: str) -> np.ndarray:
    """A BK group as int64 ns (each fraction times the 10 ms unit)."""
    rows = []
    for t in PAPER_BENCHMARKS[name]:
        rows.append([int(round(f * PAPER_UNIT_NS)) for f in PAPER_TASKS_UNITS[t]])
    return np.asarray(rows, dtype=np.int64)


def rounds_experiment(benchmark: str, workers: int, rounds: int, seed: int) -> np.ndarray:
    """Section 6.2 experiment: workers x rounds tasks drawn uniformly (with
    replacement) from the four tasks of a BK benchmark; task (w, r) at row
    w * rounds + r."""
    base = paper_benchmark(benchmark)
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.integers(0, len(base), size=workers * rounds)
    return np.ascontiguousarray(base[idx])


# Host-to-device copy rate used to turn transfer times into buffer sizes
# (about 57 GB/s, pinned-memory copies measured on the target).
FOOTPRINT_BYTES_PER_NS = 57.0


def footprints(tasks, bytes_per_ns: float = FOOTPRINT_BYTES_PER_NS) -> np.ndarray:
    """Device-memory footprint of each task (int64 bytes): its input and
    output buffers, sized from its HtD and DtH times at ``bytes_per_ns``."""
    t = np.asarray(tasks, dtype=np.int64).reshape(-1, 3)
    return np.rint((t[:, 0] + t[:, 2]).astype(np.float64) * bytes_per_ns).astype(np.int64)


def capacity_fraction(mem, frac: float) -> int:
    """A capacity of ``frac`` of the group's total footprint, never below the
    largest single footprint (every task must fit alone) nor below 1."""
    m = np.asarray(mem, dtype=np.int64)
    return int(max(1, int(m.max(initial=0)), int(math.floor(float(m.sum()) * frac))))
