"""Plain, slow CPU oracle of the temporal execution model and the ordering heuristic.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark; never by the product path.  Shares no code with the
HIP library.

What is modelled (Section 3.2 launch schemes, Section 4.1 simulator,
Section 4.2 command-time estimation):

* A task is three commands executed in order: HtD transfer, kernel K, DtH
  transfer (Section 3; a transfer stage may be empty -- zero duration).
* The simulator keeps one FIFO software queue per command type, filled in the
  launch ordering.  A head command starts when its engine is free and its
  intra-task predecessor has completed (Section 4.1, figure of the FIFO model).
  Two-DMA devices run HtD, K and DtH on three engines (three command queues);
  one-DMA devices run every transfer on one engine, all HtD before any DtH
  (Section 3.2, launch-scheme figures).
* There is a single kernel queue: kernels never run concurrently and a kernel
  always takes its solo time (Section 4.1, last paragraph; Section 4.2.2).
* At each simulation step the ready heads are started, their end times
  estimated, and time jumps to the earliest end (Section 4.1, simulation
  timeline figure).  When an HtD and a DtH run at the same time their end times
  are re-estimated from the overlap (Section 4.2.1).  The paper gives no
  formula; the reading used here: while both directions are busy, HtD advances
  at p_htd/q and DtH at p_dth/q of its solo speed, otherwise at full speed.
* Integer mode (the normative one): remaining transfer work is kept exactly in
  units of 1/q solo-nanosecond; a completion estimate is rounded up to whole
  nanoseconds.  Exact mode uses ``fractions.Fraction`` and never rounds.

Rank convention: lexicographic; rank 0 is the identity ordering.  Ties in the
best/worst ordering go to the lowest rank.
"""
from __future__ import annotations

import itertools
import math
from collections import deque
from dataclasses import dataclass
from fractions import Fraction

HTD, KER, DTH = "HtD", "K", "DtH"


@dataclass(frozen=True)
class Model:
    """Model parameters: DMA engine count and the overlap rates p/q."""

    q: int = 4
    p_htd: int = 3
    p_dth: int = 3
    dma_engines: int = 2

    def __post_init__(self):
        if self.dma_engines not in (1, 2):
            raise ValueError("dma_engines must be 1 or 2")
        if self.q < 1 or not (1 <= self.p_htd <= self.q) or not (1 <= self.p_dth <= self.q):
            raise ValueError("rates must satisfy 1 <= p <= q")


# Benchmark default: overlapped transfers each keep 3/4 of their solo speed.
DEFAULT = Model(4, 3, 3, 2)
# Rates reconstructed from the worked timeline of Section 4.1 (3/8 each).
PAPER_EXAMPLE = Model(8, 3, 3, 2)
# No slowdown at all: the three-machine permutation flow shop.
NO_SLOWDOWN = Model(1, 1, 1, 2)


def _ceil_div(a: int, b: int) -> int:
    return -((-a) // b)


def simulate(tasks, order, model: Model = DEFAULT, exact: bool = False, trace: bool = False):
    """Predicted total time of the task group launched in ``order``.

    tasks: sequence of (h, k, d) solo durations (non-negative integers, ns).
    order: sequence of task indices (a permutation of a subset of the tasks).
    Returns T, or (T, events) when ``trace``; events maps (kind, task) to
    [start, end].  Follows Section 4.1 step by step.
    """
    q = model.q
    dur = {HTD: [int(t[0]) for t in tasks], KER: [int(t[1]) for t in tasks],
           DTH: [int(t[2]) for t in tasks]}
    order = [int(x) for x in order]
    # FIFO software queues, one per engine, filled in launch order.
    if model.dma_engines == 2:
        engines = ("E_htd", "E_k", "E_dth")
        fifo = {"E_htd": deque((HTD, x) for x in order),
                "E_k": deque((KER, x) for x in order),
                "E_dth": deque((DTH, x) for x in order)}
    else:
        engines = ("E_xfer", "E_k")
        fifo = {"E_xfer": deque([(HTD, x) for x in order] + [(DTH, x) for x in order]),
                "E_k": deque((KER, x) for x in order)}
    running = {e: None for e in engines}  # the command at the head, once started
    left = {e: 0 for e in engines}  # transfers: 1/q solo-ns of work; kernel: ns
    finished = set()
    events = {}
    t = Fraction(0) if exact else 0

    def is_ready(cmd):
        kind, x = cmd
        if kind == HTD:
            return True
        if kind == KER:
            return (HTD, x) in finished
        return (KER, x) in finished

    while True:
        # At the current instant: retire what has completed and start every
        # ready head, until nothing changes (zero-length commands chain here).
        changed = True
        while changed:
            changed = False
            for e in engines:
                if running[e] is not None and left[e] == 0:
                    finished.add(running[e])
                    events[running[e]][1] = t
                    running[e] = None
                    changed = True
            for e in engines:
                if running[e] is None and fifo[e] and is_ready(fifo[e][0]):
                    cmd = fifo[e].popleft()
                    kind, x = cmd
                    running[e] = cmd
                    left[e] = dur[kind][x] * (1 if kind == KER else q)
                    events[cmd] = [t, None]
                    changed = True
        busy = [e for e in engines if running[e] is not None]
        if not busy:
            assert all(not fifo[e] for e in engines), "deadlock: commands left unstarted"
            break
        # Transfer speed: slowed down while both directions are moving data.
        kinds = {running[e][0] for e in busy}
        overlap = HTD in kinds and DTH in kinds
        rate = {}
        for e in busy:
            kind = running[e][0]
            if kind == KER:
                rate[e] = 1
            elif overlap:
                rate[e] = model.p_htd if kind == HTD else model.p_dth
            else:
                rate[e] = q
        # End-time estimates of the running commands; advance to the earliest.
        est = {e: (Fraction(left[e], rate[e]) if exact else _ceil_div(left[e], rate[e])) for e in busy}
        delta = min(est.values())
        t = t + delta
        for e in busy:
            if est[e] == delta:
                left[e] = 0
            else:
                left[e] = left[e] - rate[e] * delta
    total = max((v[1] for v in events.values()), default=0)
    if trace:
        return total, events
    return total


def update(tasks, ot, model: Model = DEFAULT):
    """Completion times (t_HtD, t_K, t_DtH) of the last ordered task when the
    ordered set OT is simulated on its own (Algorithm 1, ``update``)."""
    _, ev = simulate(tasks, ot, model, trace=True)
    last = ot[-1]
    return ev[(HTD, last)][1], ev[(KER, last)][1], ev[(DTH, last)][1]


# ----------------------------------------------------------------- enumeration

def lehmer_rank(perm) -> int:
    """Lexicographic rank: sum over positions of (#later smaller) * (n-1-i)!."""
    n = len(perm)
    r = 0
    for i in range(n):
        c = sum(1 for j in range(i + 1, n) if perm[j] < perm[i])
        r += c * math.factorial(n - 1 - i)
    return r


def all_times(tasks, model: Model = DEFAULT):
    """T for every ordering, indexed by lexicographic rank.

    itertools.permutations of range(n) yields orderings in lexicographic
    order, so the enumeration index is the rank.
    """
    n = len(tasks)
    return [simulate(tasks, p, model) for p in itertools.permutations(range(n))]


FP_MASK = (1 << 64) - 1


def summarize(times, n):
    """Best/worst/average over all orderings (the paper's speedups are taken
    against the worst ordering and reported beside the best and the average).

    fingerprint = sum over ranks r of (2r + 1) * T_r, modulo 2**64.
    """
    best = min(range(len(times)), key=lambda r: (times[r], r))
    worst = min(range(len(times)), key=lambda r: (-times[r], r))
    s = sum(times)
    fp = 0
    for r, t in enumerate(times):
        fp = (fp + (2 * r + 1) * t) & FP_MASK
    perms = None
    return {
        "min_ns": times[best], "argmin_rank": best,
        "max_ns": times[worst], "argmax_rank": worst,
        "sum": s, "count": len(times), "mean_ns": s / len(times),
        "fingerprint": fp,
        "best": list(nth_permutation(n, best)), "worst": list(nth_permutation(n, worst)),
    }


def nth_permutation(n: int, r: int):
    """The r-th ordering in lexicographic order (walks itertools' order for small n)."""
    if n <= 8:
        return next(itertools.islice(itertools.permutations(range(n)), r, None))
    # Larger n: pick, position by position, the element whose block holds r.
    rest = list(range(n))
    out = []
    for i in range(n):
        block = math.factorial(n - 1 - i)
        c, r = divmod(r, block)
        out.append(rest.pop(c))
    return tuple(out)


def exhaustive(tasks, model: Model = DEFAULT):
    times = all_times(tasks, model)
    s = summarize(times, len(tasks))
    s["times"] = times
    return s


# ------------------------------------------------------------------ heuristic
# Algorithm 1 (Section 5.1).  The paper describes the three selection
# functions only in words; the readings used:
#   select_first : the task with the largest K - HtD (short HtD, long K);
#                  ties go to the longer DtH, then the lower index.
#   select_next  : the candidate c minimising
#                  |h_c - (t_K - t_HtD)| + |k_c - (t_DtH - max(t_HtD + h_c, t_K))|,
#                  i.e. its HtD best fills the kernel engine's remaining busy
#                  time and its kernel best fills the DtH engine's remaining
#                  busy time; ties go to the lower index.
#   select_last  : for both orders (x, y) of the last two tasks, the score
#                  fit(x | OT) + fit(y | OT + x) + d_y; the smaller wins, ties
#                  go to the shorter final DtH, then to x with lower index.
# t_HtD, t_K, t_DtH always come from simulating OT alone (``update``).

def _fit(task, t_h, t_k, t_d):
    h, k, _ = task
    return abs(h - (t_k - t_h)) + abs(k - (t_d - max(t_h + h, t_k)))


def select_first(tasks, rt):
    best = None
    for c in rt:
        h, k, d = tasks[c]
        key = (-(k - h), -d, c)
        if best is None or key < best[0]:
            best = (key, c)
    return best[1]


def select_next(tasks, rt, t_h, t_k, t_d):
    best = None
    for c in rt:
        f = _fit(tasks[c], t_h, t_k, t_d)
        if best is None or f < best[0]:
            best = (f, c)
    return best[1]


def select_last(tasks, rt, ot, model, update_fn=None):
    update_fn = update_fn or update
    a, b = sorted(rt)
    t_h, t_k, t_d = update_fn(tasks, ot, model)
    best = None
    for x, y in ((a, b), (b, a)):
        s1 = _fit(tasks[x], t_h, t_k, t_d)
        u_h, u_k, u_d = update_fn(tasks, ot + [x], model)
        s2 = _fit(tasks[y], u_h, u_k, u_d)
        key = (s1 + s2 + int(tasks[y][2]), int(tasks[y][2]))
        if best is None or key < best[0]:
            best = (key, [x, y])
    return best[1]


def heuristic(tasks, model: Model = DEFAULT, update_fn=None):
    """Ordering chosen by Algorithm 1 (under the readings above).  update_fn
    (default ``update``) simulates the ordered set alone."""
    update_fn = update_fn or update
    tasks = [tuple(int(v) for v in t) for t in tasks]
    n = len(tasks)
    if n == 0:
        return []
    rt = list(range(n))
    ot = []
    first = select_first(tasks, rt)
    ot.append(first)
    rt.remove(first)
    if len(rt) == 0:
        return ot
    t_h, t_k, t_d = update_fn(tasks, ot, model)
    while len(rt) > 2:
        nxt = select_next(tasks, rt, t_h, t_k, t_d)
        ot.append(nxt)
        rt.remove(nxt)
        t_h, t_k, t_d = update_fn(tasks, ot, model)
    if len(rt) == 2:
        ot += select_last(tasks, rt, ot, model, update_fn)
    else:
        ot.append(rt[0])
    return ot


def dominant_kernel(task) -> bool:
    """DK if HtD + DtH <= K, else DT (Section 4.3)."""
    h, k, d = task
    return h + d <= k
