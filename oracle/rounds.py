"""CPU oracle for multi-round task groups (Section 6.2): T workers, each
offloading R dependent tasks.  A worker hands over its next task only when
its previous one has completely finished (its DtH has ended).

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's CPU
baseline use this module; the library never imports it.

Task (w, r) is worker w's r-th task; it is stored at index w * R + r of the
flat task table.  The device model is the FIFO simulator of Section 4.1 with
the overlap rates of Section 4.2.1 (same readings as ``model.simulate``),
extended with (a) commands that enter their queues at a given instant and
(b) the intra-worker dependency: the HtD of (w, r) may not start before the
DtH of (w, r - 1) has ended (an OpenCL event on an in-order queue, so the
commands queued behind it wait too).

Two setups, both from Section 6.2:

* NoReorder.  One thread submits all T*R tasks at t = 0, round by round, each
  round in a worker order pi_r.  Every combination (pi_0, ..., pi_{R-1}) is an
  ordering: (T!)^R of them, ranked lexicographically with pi_0 most
  significant and each pi_r ranked lexicographically.
* Heuristic.  A proxy thread takes every task waiting in the shared buffer as
  a task group, orders it with Algorithm 1 (``model.heuristic`` on the group's
  tasks, in ascending worker order) and submits it.  Reading: it hands HtDs to
  the transfer engine just in time, so it looks at the buffer again at the
  instant the HtD of the group's last task starts; if the buffer is empty then,
  it takes the tasks that arrive at the next arrival instant.

Launch schemes (Section 3.2): with two DMA engines each submitted group adds
its HtDs, kernels and DtHs to three FIFO queues in group order.  With one DMA
engine the group's HtDs and then its DtHs go to the one transfer queue and
its kernels to the kernel queue.  NoReorder submits one group per round.

The paper's NoReorder runs enable concurrent kernels (one queue per kernel);
the model has no concurrent-kernel rule, so both setups here keep the model's
single kernel queue.
"""
import itertools
import math
from collections import deque
from fractions import Fraction

from . import model as M

HTD, KER, DTH = M.HTD, M.KER, M.DTH


def _ceil_div(a, b):
    return -((-a) // b)


def simulate(tasks, T, R, model: M.Model = M.DEFAULT, perms=None, exact=False, trace=False):
    """Total time of T workers x R rounds.

    tasks: flat sequence of (h, k, d), task (w, r) at index w * R + r.
    perms: list of R worker orders (NoReorder), or None for the Heuristic
    setup.  Returns T, or (T, info) with ``trace``: info has the events
    {(kind, task index): [start, end]} and the submitted groups as
    (formation instant, [task indices in order]).
    """
    assert len(tasks) == T * R
    dur = {HTD: [int(t[0]) for t in tasks], KER: [int(t[1]) for t in tasks],
           DTH: [int(t[2]) for t in tasks]}
    q = model.q
    two = model.dma_engines == 2
    engines = ("E_htd", "E_k", "E_dth") if two else ("E_xfer", "E_k")
    fifo = {e: deque() for e in engines}
    running = {e: None for e in engines}
    left = {e: 0 for e in engines}
    finished = set()
    events = {}
    groups = []
    t = Fraction(0) if exact else 0

    def submit(order):
        groups.append((t, list(order)))
        if two:
            fifo["E_htd"].extend((HTD, x) for x in order)
            fifo["E_k"].extend((KER, x) for x in order)
            fifo["E_dth"].extend((DTH, x) for x in order)
        else:
            fifo["E_xfer"].extend([(HTD, x) for x in order] + [(DTH, x) for x in order])
            fifo["E_k"].extend((KER, x) for x in order)

    proxy = perms is None
    buffer = []      # task indices waiting for the proxy, in arrival order
    armed = False    # the proxy is looking at the buffer
    trigger = None   # the HtD whose start makes the proxy look again
    if proxy:
        buffer = [w * R for w in range(T)]
        armed = True
    else:
        assert len(perms) == R
        for r in range(R):
            assert sorted(perms[r]) == list(range(T))
            submit([w * R + r for w in perms[r]])

    def is_ready(cmd):
        kind, x = cmd
        if kind == HTD:
            return x % R == 0 or (DTH, x - 1) in finished
        if kind == KER:
            return (HTD, x) in finished
        return (KER, x) in finished

    while True:
        changed = True
        while changed:
            changed = False
            for e in engines:
                if running[e] is not None and left[e] == 0:
                    cmd = running[e]
                    finished.add(cmd)
                    events[cmd][1] = t
                    running[e] = None
                    changed = True
                    kind, x = cmd
                    if proxy and kind == DTH and x % R + 1 < R:
                        buffer.append(x + 1)  # the worker hands over its next task
            for e in engines:
                if running[e] is None and fifo[e] and is_ready(fifo[e][0]):
                    cmd = fifo[e].popleft()
                    kind, x = cmd
                    running[e] = cmd
                    left[e] = dur[kind][x] * (1 if kind == KER else q)
                    events[cmd] = [t, None]
                    changed = True
                    if cmd == trigger:
                        armed = True
            if proxy and armed and buffer:
                members = sorted(buffer)
                sub = [tasks[x] for x in members]
                order = [members[i] for i in M.heuristic(sub, model)]
                buffer = []
                armed = False
                trigger = (HTD, order[-1])
                submit(order)
                changed = True
        busy = [e for e in engines if running[e] is not None]
        if not busy:
            assert all(not fifo[e] for e in engines), "deadlock: commands left unstarted"
            assert not buffer, "tasks left in the buffer"
            break
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
        est = {e: (Fraction(left[e], rate[e]) if exact else _ceil_div(left[e], rate[e])) for e in busy}
        delta = min(est.values())
        t = t + delta
        for e in busy:
            if est[e] == delta:
                left[e] = 0
            else:
                left[e] = left[e] - rate[e] * delta
    assert len(finished) == 3 * T * R
    total = max((v[1] for v in events.values()), default=0)
    if trace:
        return total, {"events": events, "groups": groups}
    return total


def orderings(T, R):
    """All NoReorder orderings in rank order."""
    return itertools.product(itertools.permutations(range(T)), repeat=R)


def rank(perms, T):
    """Rank of (pi_0, ..., pi_{R-1}): mixed radix T!, pi_0 most significant."""
    f = math.factorial(T)
    r = 0
    for p in perms:
        r = r * f + M.lehmer_rank(p)
    return r


def unrank(T, R, r):
    f = math.factorial(T)
    out = []
    for _ in range(R):
        r, d = divmod(r, f)
        out.append(tuple(M.nth_permutation(T, d)))
    return out[::-1]


def noreorder_times(tasks, T, R, model: M.Model = M.DEFAULT):
    """T for every NoReorder ordering, indexed by rank."""
    return [simulate(tasks, T, R, model, perms=list(p)) for p in orderings(T, R)]


def noreorder_summary(tasks, T, R, model: M.Model = M.DEFAULT):
    """Best/worst/average over every NoReorder ordering (same fields and
    tie rules as ``model.summarize``; best/worst as per-round orders)."""
    times = noreorder_times(tasks, T, R, model)
    best = min(range(len(times)), key=lambda r: (times[r], r))
    worst = min(range(len(times)), key=lambda r: (-times[r], r))
    fp = 0
    for r, v in enumerate(times):
        fp = (fp + (2 * r + 1) * v) & M.FP_MASK
    return {
        "min_ns": times[best], "argmin_rank": best, "max_ns": times[worst], "argmax_rank": worst,
        "sum": sum(times), "count": len(times), "mean_ns": sum(times) / len(times),
        "fingerprint": fp, "best_perms": unrank(T, R, best), "worst_perms": unrank(T, R, worst),
        "times": times,
    }


def heuristic_setup(tasks, T, R, model: M.Model = M.DEFAULT):
    """Total time and submitted groups of the Heuristic setup."""
    total, info = simulate(tasks, T, R, model, perms=None, trace=True)
    return total, info["groups"]
