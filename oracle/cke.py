"""CPU oracle for task groups whose kernels may run concurrently (CKE).

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's CPU
baseline use this module; the library never imports it.

The paper keeps one kernel queue: kernels never overlap (Section 4.1, last
paragraph), because a kernel that exhausts the device's resources overlaps
the next one only at its tail and because the devices do not disclose how
they run concurrent kernels; its NoReorder experiments do run with one
command queue per kernel (Section 6.2), and its conclusion names concurrent
kernels as future work.  Section 3.2 gives the condition for overlap: kernels
from different queues can run together only while the device's computing
resources are not exhausted.  The reading modelled here:

* The device has ``capacity`` units of computing resources (for instance its
  compute units).  Kernel x holds units[x] of them (1 .. capacity) from its
  start to its end; a kernel that exhausts the device holds all of them.
* Kernels are dispatched in launch order (one queue per kernel, taken in
  submission order by the device): K_x starts as soon as its HtD has ended,
  every kernel launched before it has started, and the units held by the
  running kernels plus its own fit in the capacity.  A running kernel takes
  its solo time; concurrent kernels do not slow each other down.
* Transfers are those of ``model.simulate``: FIFO queues in launch order (two
  DMA engines: HtD queue and DtH queue; one DMA engine: every HtD, then every
  DtH, on one queue), DtH_x after K_x and after the DtH before it, the
  Section 4.2.1 overlap rates, integer or exact time.
* With every kernel holding the whole capacity this is ``model.simulate``.

Algorithm 1 is unchanged; its ``update`` simulates the ordered set under the
same rule.
"""
from __future__ import annotations

import itertools
from collections import deque
from fractions import Fraction

from . import model as M

HTD, KER, DTH = M.HTD, M.KER, M.DTH


def _ceil_div(a, b):
    return -((-a) // b)


def check(tasks, units, capacity):
    if capacity < 1:
        raise ValueError("capacity must be at least 1")
    if len(units) != len(tasks):
        raise ValueError("one unit count per task")
    for u in units:
        if u < 1 or u > capacity:
            raise ValueError("every kernel needs 1..capacity units")


def simulate(tasks, units, capacity, order, model: M.Model = M.DEFAULT, exact=False, trace=False):
    """Predicted total time of ``order`` under the CKE reading above.
    Returns T, or (T, events) when ``trace`` (events maps (kind, task) to
    [start, end])."""
    units = [int(u) for u in units]
    check(tasks, units, capacity)
    q = model.q
    dur = {HTD: [int(t[0]) for t in tasks], KER: [int(t[1]) for t in tasks],
           DTH: [int(t[2]) for t in tasks]}
    order = [int(x) for x in order]
    if model.dma_engines == 2:
        xfer = {"E_htd": deque((HTD, x) for x in order), "E_dth": deque((DTH, x) for x in order)}
    else:
        xfer = {"E_xfer": deque([(HTD, x) for x in order] + [(DTH, x) for x in order])}
    kq = deque(order)                 # kernels waiting for dispatch, launch order
    running = {e: None for e in xfer}  # transfer at the head of each engine, once started
    left = {e: 0 for e in xfer}        # its remaining work, 1/q solo-ns
    kleft = {}                         # running kernels: task -> ns left
    held = 0                           # units held by running kernels
    finished = set()
    events = {}
    t = Fraction(0) if exact else 0

    def ready(cmd):
        kind, x = cmd
        return kind == HTD or (KER, x) in finished

    while True:
        changed = True
        while changed:
            changed = False
            for e in xfer:
                if running[e] is not None and left[e] == 0:
                    finished.add(running[e])
                    events[running[e]][1] = t
                    running[e] = None
                    changed = True
            for x in [x for x, v in kleft.items() if v == 0]:
                del kleft[x]
                held -= units[x]
                finished.add((KER, x))
                events[(KER, x)][1] = t
                changed = True
            for e in xfer:
                if running[e] is None and xfer[e] and ready(xfer[e][0]):
                    cmd = xfer[e].popleft()
                    running[e] = cmd
                    left[e] = dur[cmd[0]][cmd[1]] * q
                    events[cmd] = [t, None]
                    changed = True
            # in-order dispatch: the head kernel starts once its HtD has ended
            # and its units fit beside the running kernels; those behind it wait
            while kq and (HTD, kq[0]) in finished and held + units[kq[0]] <= capacity:
                x = kq.popleft()
                kleft[x] = dur[KER][x]
                held += units[x]
                events[(KER, x)] = [t, None]
                changed = True
        busy = [e for e in xfer if running[e] is not None]
        if not busy and not kleft:
            assert not kq and all(not v for v in xfer.values()), "deadlock: commands left unstarted"
            break
        kinds = {running[e][0] for e in busy}
        overlap = HTD in kinds and DTH in kinds
        rate = {}
        for e in busy:
            kind = running[e][0]
            rate[e] = (model.p_htd if kind == HTD else model.p_dth) if overlap else q
        est = {e: (Fraction(left[e], rate[e]) if exact else _ceil_div(left[e], rate[e])) for e in busy}
        cands = list(est.values()) + list(kleft.values())
        delta = min(cands)
        t = t + delta
        for e in busy:
            left[e] = 0 if est[e] == delta else left[e] - rate[e] * delta
        for x in kleft:
            kleft[x] = kleft[x] - delta
    total = max((v[1] for v in events.values()), default=0)
    if trace:
        return total, events
    return total


def update(tasks, units, capacity, ot, model: M.Model = M.DEFAULT):
    """(t_HtD, t_K, t_DtH) of the last task of OT, OT simulated alone under CKE."""
    _, ev = simulate(tasks, units, capacity, ot, model, trace=True)
    last = ot[-1]
    return ev[(HTD, last)][1], ev[(KER, last)][1], ev[(DTH, last)][1]


def heuristic(tasks, units, capacity, model: M.Model = M.DEFAULT):
    """Algorithm 1 with ``update`` under the CKE rule."""
    units = [int(u) for u in units]
    return M.heuristic(tasks, model,
                       update_fn=lambda ts, ot, m: update(ts, units, capacity, ot, m))


def all_times(tasks, units, capacity, model: M.Model = M.DEFAULT):
    """T for every ordering, indexed by lexicographic rank."""
    n = len(tasks)
    return [simulate(tasks, units, capacity, p, model) for p in itertools.permutations(range(n))]


def exhaustive(tasks, units, capacity, model: M.Model = M.DEFAULT):
    times = all_times(tasks, units, capacity, model)
    s = M.summarize(times, len(tasks))
    s["times"] = times
    h = heuristic(tasks, units, capacity, model)
    s["heur"] = h
    s["heur_ns"] = simulate(tasks, units, capacity, h, model)
    return s
