"""CPU oracle for task groups under a device-memory limit.

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's CPU
baseline use this module; the library never imports it.

Section 5 (end) notes that tasks running concurrently hold device memory for
their inputs and outputs at the same time, so the memory available can limit
which tasks may form a task group; the paper leaves this out and assumes
enough memory.  The reading modelled here:

* Task x needs mem[x] bytes of device memory (its input and output buffers).
  They are taken when its HtD starts and given back when its DtH ends.  At
  most ``capacity`` bytes are held at any instant.
* Two DMA engines (three FIFO queues): the HtD at the head of its queue
  starts only when the bytes held plus its own fit in the capacity; the HtDs
  queued behind it wait too (in-order queue).  DtHs end in launch order, so
  the wait always ends as long as every task fits on its own.
* One DMA engine: the single transfer queue holds a group's HtDs before its
  DtHs, so a group whose buffers do not all fit would never progress.  The
  launch ordering is therefore cut greedily into consecutive sub-groups, each
  as long as its tasks fit together, and each sub-group is launched with the
  one-DMA scheme (its HtDs, then its DtHs) behind the previous one.
* Everything else is the model of ``model.simulate`` (Section 4.1 FIFO
  simulator with the Section 4.2.1 overlap rates, integer or exact mode).

Algorithm 1 is unchanged; its ``update`` simulates the ordered set under the
same memory rule (the heuristic sees the device only through ``update``).
"""
from __future__ import annotations

import itertools
from collections import deque
from fractions import Fraction

from . import model as M

HTD, KER, DTH = M.HTD, M.KER, M.DTH


def _ceil_div(a, b):
    return -((-a) // b)


def subgroups(mem, capacity, order):
    """One-DMA launch groups: consecutive runs of ``order``, each run as long
    as the buffers of its tasks fit together."""
    out = []
    cur, held = [], 0
    for x in order:
        if cur and held + mem[x] > capacity:
            out.append(cur)
            cur, held = [], 0
        cur.append(x)
        held += mem[x]
    if cur:
        out.append(cur)
    return out


def check(tasks, mem, capacity):
    if capacity <= 0:
        raise ValueError("capacity must be positive")
    if len(mem) != len(tasks):
        raise ValueError("one footprint per task")
    for m in mem:
        if m < 0 or m > capacity:
            raise ValueError("every task must fit in the capacity on its own")


def simulate(tasks, mem, capacity, order, model: M.Model = M.DEFAULT, exact=False, trace=False):
    """Total time of the group launched in ``order`` under the memory limit.

    Returns T, or (T, info) with ``trace``: info["events"] maps (kind, task)
    to [start, end]; info["groups"] lists the launch groups (one for two DMA
    engines)."""
    mem = [int(m) for m in mem]
    check(tasks, mem, capacity)
    q = model.q
    dur = {HTD: [int(t[0]) for t in tasks], KER: [int(t[1]) for t in tasks],
           DTH: [int(t[2]) for t in tasks]}
    order = [int(x) for x in order]
    if model.dma_engines == 2:
        groups = [order]
        engines = ("E_htd", "E_k", "E_dth")
        fifo = {"E_htd": deque((HTD, x) for x in order),
                "E_k": deque((KER, x) for x in order),
                "E_dth": deque((DTH, x) for x in order)}
    else:
        groups = subgroups(mem, capacity, order)
        engines = ("E_xfer", "E_k")
        xfer = deque()
        for g in groups:
            xfer.extend((HTD, x) for x in g)
            xfer.extend((DTH, x) for x in g)
        fifo = {"E_xfer": xfer, "E_k": deque((KER, x) for x in order)}
    running = {e: None for e in engines}
    left = {e: 0 for e in engines}
    finished = set()
    events = {}
    held = 0
    t = Fraction(0) if exact else 0

    def is_ready(cmd):
        kind, x = cmd
        if kind == HTD:
            return held + mem[x] <= capacity
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
                    if cmd[0] == DTH:
                        held -= mem[cmd[1]]        # buffers given back
            for e in engines:
                if running[e] is None and fifo[e] and is_ready(fifo[e][0]):
                    cmd = fifo[e].popleft()
                    kind, x = cmd
                    if kind == HTD:
                        held += mem[x]             # buffers taken
                    running[e] = cmd
                    left[e] = dur[kind][x] * (1 if kind == KER else q)
                    events[cmd] = [t, None]
                    changed = True
        busy = [e for e in engines if running[e] is not None]
        if not busy:
            assert all(not fifo[e] for e in engines), "deadlock: commands left unstarted"
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
    assert held == 0
    total = max((v[1] for v in events.values()), default=0)
    if trace:
        return total, {"events": events, "groups": groups}
    return total


def update(tasks, mem, capacity, ot, model: M.Model = M.DEFAULT):
    """(t_HtD, t_K, t_DtH) of the last task of OT, OT simulated alone under
    the memory limit."""
    _, info = simulate(tasks, mem, capacity, ot, model, trace=True)
    ev = info["events"]
    last = ot[-1]
    return ev[(HTD, last)][1], ev[(KER, last)][1], ev[(DTH, last)][1]


def heuristic(tasks, mem, capacity, model: M.Model = M.DEFAULT):
    """Algorithm 1 with ``update`` under the memory limit."""
    mem = [int(m) for m in mem]
    return M.heuristic(tasks, model,
                       update_fn=lambda ts, ot, m: update(ts, mem, capacity, ot, m))


def all_times(tasks, mem, capacity, model: M.Model = M.DEFAULT):
    """T for every ordering, indexed by lexicographic rank."""
    n = len(tasks)
    return [simulate(tasks, mem, capacity, p, model) for p in itertools.permutations(range(n))]


def exhaustive(tasks, mem, capacity, model: M.Model = M.DEFAULT):
    times = all_times(tasks, mem, capacity, model)
    s = M.summarize(times, len(tasks))
    s["times"] = times
    h = heuristic(tasks, mem, capacity, model)
    s["heur"] = h
    s["heur_ns"] = simulate(tasks, mem, capacity, h, model)
    return s
