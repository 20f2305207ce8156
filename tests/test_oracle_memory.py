"""Pins of the device-memory-limit oracle (task buffers held from HtD start
to DtH end, at most a capacity at once) against hand-worked timelines, the
unconstrained model it must reduce to, closed forms (fully serial execution;
the flow-shop recurrence with memory release times) and invariants."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import cmodel
from oracle import memory as MM
from oracle import model as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MODELS = [M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN, M.Model(16, 9, 13), M.Model(4, 3, 3, 1)]


def rand_case(rng, n, hi=60, mhi=10):
    tasks = [tuple(int(v) for v in rng.integers(0, hi, size=3)) for _ in range(n)]
    mem = [int(v) for v in rng.integers(0, mhi, size=n)]
    lo = max(1, max(mem))
    cap = int(rng.integers(lo, max(lo, sum(mem)) + 2))
    return tasks, mem, cap


def test_hand_worked_timelines():
    g = json.load(open(os.path.join(GOLDEN, "memory_hand.json")))
    for case in g["cases"]:
        m = M.Model(**case["model"])
        T, info = MM.simulate(g["tasks_ns"], g["mem"], case["capacity"], case["order"], m, trace=True)
        assert T == case["T"]
        assert info["groups"] == case["groups"]
        assert {f"{k}_{x}": v for (k, x), v in info["events"].items()} == case["events"]
        Te = MM.simulate(g["tasks_ns"], g["mem"], case["capacity"], case["order"], m, exact=True)
        assert Te == Fraction(case["T_exact"])


def test_enough_memory_is_the_unconstrained_model():
    rng = np.random.default_rng(60)
    for _ in range(40):
        n = int(rng.integers(1, 6))
        tasks, mem, _ = rand_case(rng, n)
        cap = max(1, sum(mem))
        for m in MODELS:
            for p in itertools.permutations(range(n)):
                assert MM.simulate(tasks, mem, cap, p, m) == M.simulate(tasks, p, m)
            assert MM.heuristic(tasks, mem, cap, m) == M.heuristic(tasks, m)


def test_one_task_at_a_time_is_serial():
    # every pair of footprints exceeds the capacity: no two tasks are ever
    # resident together, so the group runs back to back whatever the order
    rng = np.random.default_rng(61)
    for _ in range(40):
        n = int(rng.integers(1, 6))
        tasks = [tuple(int(v) for v in rng.integers(0, 60, size=3)) for _ in range(n)]
        mem = [int(v) for v in rng.integers(51, 101, size=n)]
        serial = sum(sum(t) for t in tasks)
        for m in MODELS:
            for p in itertools.permutations(range(n)):
                assert MM.simulate(tasks, mem, 100, p, m) == serial


def release_flow_shop(tasks, mem, cap, order):
    """Two DMA engines at full speed: the three-machine flow-shop recurrence,
    the HtD at position j released by the end of the DtH at position a_j - 1,
    a_j the first position from which the footprints through j fit."""
    He, Ke, De = [], [], []
    for j, x in enumerate(order):
        a = j
        while a > 0 and sum(mem[order[i]] for i in range(a - 1, j + 1)) <= cap:
            a -= 1
        h, k, d = tasks[x]
        start = max(He[-1] if He else 0, De[a - 1] if a > 0 else 0)
        He.append(start + h)
        Ke.append(max(He[-1], Ke[-1] if Ke else 0) + k)
        De.append(max(Ke[-1], De[-1] if De else 0) + d)
    return De[-1] if De else 0


def one_dma_chain(tasks, mem, cap, order):
    """One DMA engine (no overlap slowdown): per greedy sub-group, its HtDs
    back to back, then its DtHs, on one engine; kernels in order on another."""
    X = 0        # transfer engine free
    Kprev = 0
    b = 0
    n = len(order)
    while b < n:
        e, held = b, 0
        while e < n and (e == b or held + mem[order[e]] <= cap):
            held += mem[order[e]]
            e += 1
        H, K = [], []
        for x in order[b:e]:
            X += tasks[x][0]
            H.append(X)
            Kprev = max(X, Kprev) + tasks[x][1]
            K.append(Kprev)
        D = X
        for i, x in enumerate(order[b:e]):
            D = max(K[i], D) + tasks[x][2]
        X = D
        b = e
    return X


def test_closed_forms():
    rng = np.random.default_rng(62)
    for _ in range(60):
        n = int(rng.integers(1, 6))
        tasks, mem, cap = rand_case(rng, n)
        for p in itertools.permutations(range(n)):
            assert MM.simulate(tasks, mem, cap, p, M.NO_SLOWDOWN) == release_flow_shop(tasks, mem, cap, p)
            for m in (M.Model(4, 3, 3, 1), M.Model(8, 1, 5, 1)):   # one engine: rates never apply
                assert MM.simulate(tasks, mem, cap, p, m) == one_dma_chain(tasks, mem, cap, p)


def test_more_memory_never_hurts_without_slowdown():
    # max-plus recurrence: larger capacity only moves release times earlier
    rng = np.random.default_rng(63)
    for _ in range(30):
        n = int(rng.integers(2, 6))
        tasks, mem, _ = rand_case(rng, n)
        caps = sorted({max(1, max(mem)) + i for i in range(sum(mem) + 1)})
        for p in itertools.permutations(range(n)):
            ts = [MM.simulate(tasks, mem, c, p, M.NO_SLOWDOWN) for c in caps]
            assert all(a >= b for a, b in zip(ts, ts[1:]))


def test_trace_invariants():
    rng = np.random.default_rng(64)
    for _ in range(60):
        n = int(rng.integers(1, 7))
        tasks, mem, cap = rand_case(rng, n, 40)
        for m in MODELS:
            order = [int(v) for v in rng.permutation(n)]
            T, info = MM.simulate(tasks, mem, cap, order, m, trace=True)
            ev = info["events"]
            for x in range(n):
                h, k, d = (ev[(kd, x)] for kd in (M.HTD, M.KER, M.DTH))
                assert h[0] <= h[1] <= k[0] <= k[1] <= d[0] <= d[1] <= T
                assert k[1] - k[0] == tasks[x][1]
                assert h[1] - h[0] >= tasks[x][0] and d[1] - d[0] >= tasks[x][2]
            # held bytes at every instant (intervals [HtD start, DtH end))
            for t in {v[0] for v in ev.values()}:
                held = sum(mem[x] for x in range(n)
                           if ev[(M.HTD, x)][0] <= t < ev[(M.DTH, x)][1] or
                           ev[(M.HTD, x)][0] == t == ev[(M.DTH, x)][1])
                assert held <= cap
            # engines in launch order
            groups = info["groups"]
            assert [x for g in groups for x in g] == order
            queues = ([[(kd, x) for x in order] for kd in (M.HTD, M.KER, M.DTH)] if m.dma_engines == 2 else
                      [[(kd, x) for g in groups for kd in (M.HTD, M.DTH) for x in g],
                       [(M.KER, x) for x in order]])
            for qu in queues:
                for a, b in zip(qu, qu[1:]):
                    assert ev[a][1] <= ev[b][0]
            if m.dma_engines == 1:
                # maximal sub-groups: each fits, and the next task would not
                for i, g in enumerate(groups):
                    assert sum(mem[x] for x in g) <= cap
                    if i + 1 < len(groups):
                        assert sum(mem[x] for x in g) + mem[groups[i + 1][0]] > cap
            else:
                assert groups == [order]


def test_lower_bounds():
    rng = np.random.default_rng(65)
    for _ in range(60):
        n = int(rng.integers(1, 6))
        tasks, mem, cap = rand_case(rng, n)
        for m in MODELS:
            order = [int(v) for v in rng.permutation(n)]
            T = MM.simulate(tasks, mem, cap, order, m)
            assert T >= max(sum(t[0] for t in tasks), sum(t[1] for t in tasks), sum(t[2] for t in tasks))
            if m.dma_engines == 2:
                # each command starts no earlier and lasts no shorter than in
                # the unconstrained flow shop at full speed
                assert T >= M.simulate(tasks, order, M.NO_SLOWDOWN)
            else:
                assert T >= sum(t[0] + t[2] for t in tasks)


def test_integer_within_rounding_bound_of_exact():
    rng = np.random.default_rng(66)
    for _ in range(60):
        n = int(rng.integers(1, 6))
        tasks, mem, cap = rand_case(rng, n, 1000)
        for m in (M.DEFAULT, M.PAPER_EXAMPLE, M.Model(16, 9, 13)):
            order = [int(v) for v in rng.permutation(n)]
            Ti = MM.simulate(tasks, mem, cap, order, m)
            Te = MM.simulate(tasks, mem, cap, order, m, exact=True)
            assert abs(Ti - Te) <= 3 * n * math.ceil(m.q / min(m.p_htd, m.p_dth))


def test_heuristic_structure():
    # parity unpinned beyond structure: Algorithm 1 gives no worked example
    rng = np.random.default_rng(67)
    for _ in range(40):
        n = int(rng.integers(1, 8))
        tasks, mem, cap = rand_case(rng, n)
        for m in MODELS:
            h = MM.heuristic(tasks, mem, cap, m)
            assert sorted(h) == list(range(n))
            assert h[0] == M.select_first(tasks, list(range(n)))


def test_input_checks():
    with pytest.raises(ValueError):
        MM.simulate([(1, 1, 1)], [5], 4, [0])
    with pytest.raises(ValueError):
        MM.simulate([(1, 1, 1)], [-1], 4, [0])
    with pytest.raises(ValueError):
        MM.simulate([(1, 1, 1)], [1], 0, [0])


def test_c_transcription_matches():
    rng = np.random.default_rng(68)
    for _ in range(30):
        n = int(rng.integers(1, 7))
        tasks, mem, cap = rand_case(rng, n, 200)
        for m in MODELS:
            want = MM.all_times(tasks, mem, cap, m)
            assert list(cmodel.mem_times(tasks, mem, cap, m, threads=3)) == want
            lo, hi = len(want) // 3, len(want) // 3 + len(want) // 2
            assert list(cmodel.mem_times(tasks, mem, cap, m, lo=lo, hi=hi, threads=2)) == want[lo:hi]
