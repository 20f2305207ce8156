"""Pins of the multi-round oracle (Section 6.2: T workers x R dependent
tasks, NoReorder and Heuristic setups) against hand-worked timelines, the
single-group model it must reduce to, closed forms and invariants."""
import itertools
import json
import math
import os

import numpy as np

from oracle import cmodel
from oracle import model as M
from oracle import rounds as RD

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MODELS = [M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN, M.Model(16, 9, 13), M.Model(4, 3, 3, 1)]


def rand_tasks(rng, n, lo=0, hi=60):
    return [tuple(int(v) for v in rng.integers(lo, hi, size=3)) for _ in range(n)]


def ev_name(key):
    kind, x = key
    return f"{kind}_{x}"


def test_hand_worked_timelines():
    g = json.load(open(os.path.join(GOLDEN, "rounds_hand.json")))
    m = M.Model(**g["model"])
    for case in g["cases"]:
        T, info = RD.simulate(case["tasks_ns"], 2, 2, m, perms=case["perms"], trace=True)
        assert T == case["T"]
        got = {ev_name(k): v for k, v in info["events"].items()}
        assert got == case["events"]
    for case in g["heuristic_cases"]:
        T, info = RD.simulate(case["tasks_ns"], 2, 2, m, perms=None, trace=True)
        assert T == case["T"]
        assert [[t, o] for t, o in info["groups"]] == case["groups"]
        assert {ev_name(k): v for k, v in info["events"].items()} == case["events"]


def test_one_round_is_the_single_group_model():
    rng = np.random.default_rng(40)
    for _ in range(30):
        T = int(rng.integers(1, 6))
        tasks = rand_tasks(rng, T)
        for m in MODELS:
            for p in itertools.permutations(range(T)):
                assert RD.simulate(tasks, T, 1, m, perms=[p]) == M.simulate(tasks, p, m)
            h, groups = RD.heuristic_setup(tasks, T, 1, m)
            assert len(groups) == 1 and groups[0][1] == M.heuristic(tasks, m)
            assert h == M.simulate(tasks, M.heuristic(tasks, m), m)


def test_one_worker_runs_its_tasks_back_to_back():
    # only one task is ever in flight, so no transfer overlaps another
    rng = np.random.default_rng(41)
    for _ in range(30):
        R = int(rng.integers(1, 7))
        tasks = rand_tasks(rng, R)
        serial = sum(sum(t) for t in tasks)
        for m in MODELS:
            assert RD.simulate(tasks, 1, R, m, perms=[(0,)] * R) == serial
            assert RD.heuristic_setup(tasks, 1, R, m)[0] == serial


def check_trace(tasks, T, R, m, info, proxy):
    ev = info["events"]
    n = T * R
    assert len(ev) == 3 * n
    for x in range(n):
        h, k, d = (ev[(kind, x)] for kind in (M.HTD, M.KER, M.DTH))
        assert h[0] <= h[1] <= k[0] <= k[1] <= d[0] <= d[1]
        assert k[1] - k[0] == tasks[x][1]                       # kernels never slow down
        assert h[1] - h[0] >= tasks[x][0] and d[1] - d[0] >= tasks[x][2]
        if x % R:
            assert h[0] >= ev[(M.DTH, x - 1)][1]                # the worker's dependency
    # each engine runs one command at a time, in submission order
    seq = [x for _, order in info["groups"] for x in order]
    assert sorted(seq) == list(range(n))
    queues = ([[(M.HTD, x) for x in seq], [(M.KER, x) for x in seq], [(M.DTH, x) for x in seq]]
              if m.dma_engines == 2 else
              [[(kd, x) for _, o in info["groups"] for kd in (M.HTD, M.DTH) for x in o],
               [(M.KER, x) for x in seq]])
    for q in queues:
        for a, b in zip(q, q[1:]):
            assert ev[a][1] <= ev[b][0]
    if proxy:
        # a group holds only tasks whose predecessor had finished, and every
        # task is submitted no earlier than that
        for t0, order in info["groups"]:
            for x in order:
                assert x % R == 0 or ev[(M.DTH, x - 1)][1] <= t0
                assert ev[(M.HTD, x)][0] >= t0


def test_trace_invariants_random():
    rng = np.random.default_rng(42)
    for _ in range(60):
        T = int(rng.integers(1, 5))
        R = int(rng.integers(1, 4))
        tasks = rand_tasks(rng, T * R, 0, 40)
        for m in MODELS:
            perms = [tuple(int(v) for v in rng.permutation(T)) for _ in range(R)]
            _, info = RD.simulate(tasks, T, R, m, perms=perms, trace=True)
            check_trace(tasks, T, R, m, info, False)
            _, info = RD.simulate(tasks, T, R, m, perms=None, trace=True)
            check_trace(tasks, T, R, m, info, True)


def test_lower_bounds():
    rng = np.random.default_rng(43)
    for _ in range(80):
        T = int(rng.integers(1, 5))
        R = int(rng.integers(1, 4))
        tasks = rand_tasks(rng, T * R)
        for m in MODELS:
            perms = [tuple(int(v) for v in rng.permutation(T)) for _ in range(R)]
            for tot in (RD.simulate(tasks, T, R, m, perms=perms), RD.heuristic_setup(tasks, T, R, m)[0]):
                for w in range(T):
                    assert tot >= sum(sum(tasks[w * R + r]) for r in range(R))
                assert tot >= sum(t[0] for t in tasks) and tot >= sum(t[1] for t in tasks)
                assert tot >= sum(t[2] for t in tasks)
                if m.dma_engines == 1:
                    assert tot >= sum(t[0] + t[2] for t in tasks)


def test_relabelling_workers_permutes_orderings():
    rng = np.random.default_rng(44)
    for _ in range(8):
        T, R = 3, 2
        tasks = rand_tasks(rng, T * R)
        sigma = [int(v) for v in rng.permutation(T)]       # new label of worker w
        moved = [None] * (T * R)
        for w in range(T):
            for r in range(R):
                moved[sigma[w] * R + r] = tasks[w * R + r]
        for perms in RD.orderings(T, R):
            mp = [tuple(sigma[w] for w in p) for p in perms]
            assert RD.simulate(tasks, T, R, M.DEFAULT, perms=list(perms)) == \
                RD.simulate(moved, T, R, M.DEFAULT, perms=mp)


def test_rank_unrank_and_order():
    for T, R in ((1, 3), (2, 2), (3, 2), (2, 3), (4, 1)):
        allp = list(RD.orderings(T, R))
        assert len(allp) == math.factorial(T) ** R
        for r, p in enumerate(allp):
            assert RD.rank(p, T) == r
            assert [tuple(x) for x in RD.unrank(T, R, r)] == [tuple(x) for x in p]


def test_summary_by_brute_force():
    rng = np.random.default_rng(45)
    tasks = rand_tasks(rng, 6, 1, 1000)
    s = RD.noreorder_summary(tasks, 3, 2, M.DEFAULT)
    times = s["times"]
    assert s["count"] == 36 and s["sum"] == sum(times)
    assert s["min_ns"] == min(times) and times.index(min(times)) == s["argmin_rank"]
    assert s["max_ns"] == max(times) and times.index(max(times)) == s["argmax_rank"]
    assert s["fingerprint"] == sum((2 * r + 1) * t for r, t in enumerate(times)) % (1 << 64)
    assert RD.simulate(tasks, 3, 2, M.DEFAULT, perms=s["best_perms"]) == s["min_ns"]


def test_integer_mode_within_rounding_bound_of_exact():
    rng = np.random.default_rng(46)
    for _ in range(60):
        T = int(rng.integers(1, 4))
        R = int(rng.integers(1, 4))
        tasks = rand_tasks(rng, T * R, 0, 1000)
        for m in (M.DEFAULT, M.PAPER_EXAMPLE, M.Model(16, 9, 13)):
            perms = [tuple(int(v) for v in rng.permutation(T)) for _ in range(R)]
            Ti = RD.simulate(tasks, T, R, m, perms=perms)
            Te = RD.simulate(tasks, T, R, m, perms=perms, exact=True)
            assert abs(Ti - Te) <= 3 * T * R * math.ceil(m.q / min(m.p_htd, m.p_dth))


def test_c_transcription_matches():
    rng = np.random.default_rng(47)
    for _ in range(25):
        T = int(rng.integers(1, 5))
        R = int(rng.integers(1, 4))
        if math.factorial(T) ** R > 2000:
            continue
        tasks = rand_tasks(rng, T * R, 0, 200)
        for m in MODELS:
            want = RD.noreorder_times(tasks, T, R, m)
            got = cmodel.rounds_times(tasks, T, R, m, threads=3)
            assert list(got) == want, (T, R, m)
