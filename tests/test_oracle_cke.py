"""Pins of the concurrent-kernel oracle (oracle/cke.py) against what the
reading fixes: hand-worked timelines, the reduction to the one-kernel-queue
model, the closed form when every kernel fits at once, machine and area lower
bounds, the serial upper bound, and Algorithm 1 under the same rule."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import cke
from oracle import model as M

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MODELS = [M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN, M.Model(4, 3, 3, 1), M.Model(8, 5, 7, 2),
          M.Model(16, 9, 16, 2)]


def rand_group(rng, n, lo=0, hi=50):
    return [tuple(int(v) for v in rng.integers(lo, hi, size=3)) for _ in range(n)]


def name_of(kind, x):
    return {M.HTD: "HtD", M.KER: "K", M.DTH: "DtH"}[kind] + str(x)


def test_hand_worked_timelines():
    g = json.load(open(os.path.join(GOLDEN, "cke_hand.json")))
    m = M.Model(**g["model"])
    for case in g["cases"]:
        T, ev = cke.simulate(case["tasks"], case["units"], case["capacity"], case["order"], m, trace=True)
        assert T == case["T"], case["name"]
        got = {name_of(k, x): v for (k, x), v in ev.items()}
        assert got == case["events"], case["name"]
        if "T_one_kernel_queue" in case:
            assert M.simulate(case["tasks"], case["order"], m) == case["T_one_kernel_queue"]


def test_whole_capacity_kernels_are_the_one_queue_model():
    rng = np.random.default_rng(31)
    for m in MODELS:
        for _ in range(40):
            n = int(rng.integers(1, 7))
            tasks = rand_group(rng, n)
            C = int(rng.integers(1, 9))
            order = list(rng.permutation(n))
            assert cke.simulate(tasks, [C] * n, C, order, m) == M.simulate(tasks, order, m)
            assert cke.simulate(tasks, [C] * n, C, order, m, exact=True) == M.simulate(tasks, order, m, exact=True)


def closed_form_all_fit(tasks, order, one_dma):
    """Every kernel fits at once and transfers run at full speed: kernels start
    when their HtD ends (HtD ends grow along the ordering, so in-order
    dispatch never holds one back), then the DtH chain."""
    H = list(itertools.accumulate(int(tasks[x][0]) for x in order))
    E = [H[j] + int(tasks[x][1]) for j, x in enumerate(order)]
    D = H[-1] if one_dma else 0
    for j, x in enumerate(order):
        D = max(E[j], D) + int(tasks[x][2])
    return D


def test_closed_form_when_every_kernel_fits():
    rng = np.random.default_rng(32)
    for dma in (2, 1):
        m = M.Model(1, 1, 1, dma)
        for _ in range(60):
            n = int(rng.integers(1, 8))
            tasks = rand_group(rng, n)
            units = [int(v) for v in rng.integers(1, 4, size=n)]
            C = sum(units) + int(rng.integers(0, 3))
            order = list(rng.permutation(n))
            assert cke.simulate(tasks, units, C, order, m) == closed_form_all_fit(tasks, order, dma == 1)


def test_bounds_and_invariants():
    rng = np.random.default_rng(33)
    for m in (M.DEFAULT, M.NO_SLOWDOWN, M.Model(4, 3, 3, 1)):
        for _ in range(60):
            n = int(rng.integers(1, 7))
            tasks = rand_group(rng, n, 0, 40)
            C = int(rng.integers(1, 9))
            units = [int(v) for v in rng.integers(1, C + 1, size=n)]
            order = list(rng.permutation(n))
            T = cke.simulate(tasks, units, C, order, m)
            Tx = cke.simulate(tasks, units, C, order, m, exact=True)
            h = [t[0] for t in tasks]
            k = [t[1] for t in tasks]
            d = [t[2] for t in tasks]
            # machine bounds (transfer engines stay serial), the longest task,
            # and the kernel area: every kernel runs inside [min h, T - min d]
            lbs = [sum(h) + min(a + b for a, b in zip(k, d)), min(a + b for a, b in zip(h, k)) + sum(d),
                   max(a + b + c for a, b, c in tasks),
                   min(h) + math.ceil(Fraction(sum(a * u for a, u in zip(k, units)), C)) + min(d)]
            if m.dma_engines == 1:
                lbs.append(sum(h) + sum(d))
            assert Tx >= max(lbs) and T >= max(lbs)
            # the serial sum: overlapped transfers at p_htd + p_dth >= q never take longer than in turn
            assert Tx <= sum(h) + sum(k) + sum(d)
            # integer time: at most one ns of rounding per completion estimate of each command
            assert abs(T - Tx) <= 3 * n * math.ceil(m.q / min(m.p_htd, m.p_dth))


def test_relabelling_keeps_the_multiset_of_times():
    rng = np.random.default_rng(34)
    tasks = rand_group(rng, 5, 1, 30)
    units = [1, 3, 2, 2, 4]
    perm = [3, 0, 4, 1, 2]
    a = sorted(cke.all_times(tasks, units, 5, M.DEFAULT))
    t2 = [tasks[p] for p in perm]
    u2 = [units[p] for p in perm]
    assert a == sorted(cke.all_times(t2, u2, 5, M.DEFAULT))


def test_heuristic_under_cke():
    rng = np.random.default_rng(35)
    for _ in range(10):
        n = int(rng.integers(2, 7))
        tasks = rand_group(rng, n, 1, 40)
        C = int(rng.integers(2, 6))
        units = [int(v) for v in rng.integers(1, C + 1, size=n)]
        s = cke.exhaustive(tasks, units, C, M.DEFAULT)
        assert sorted(s["heur"]) == list(range(n))
        assert s["min_ns"] <= s["heur_ns"] <= s["max_ns"]
        # whole-capacity kernels: Algorithm 1 as in the one-queue model
        assert cke.heuristic(tasks, [C] * n, C, M.DEFAULT) == M.heuristic(tasks, M.DEFAULT)


def test_argument_checks():
    with pytest.raises(ValueError):
        cke.simulate([(1, 1, 1)], [0], 2, [0])
    with pytest.raises(ValueError):
        cke.simulate([(1, 1, 1)], [3], 2, [0])
    with pytest.raises(ValueError):
        cke.simulate([(1, 1, 1)], [1, 1], 2, [0])


def test_c_transcription_matches():
    from oracle import cmodel
    cmodel.build()
    rng = np.random.default_rng(36)
    for m in MODELS:
        for _ in range(30):
            n = int(rng.integers(1, 7))
            tasks = rand_group(rng, n)
            C = int(rng.integers(1, 9))
            units = [int(v) for v in rng.integers(1, C + 1, size=n)]
            order = list(rng.permutation(n))
            assert cmodel.cke_simulate(tasks, units, C, order, m) == cke.simulate(tasks, units, C, order, m)
        tasks = rand_group(rng, 5, 0, 30)
        units = [1, 2, 3, 2, 1]
        assert list(cmodel.cke_times(tasks, units, 3, m)) == cke.all_times(tasks, units, 3, m)
