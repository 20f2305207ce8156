"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code path: printed event
times (Section 4.1 worked timeline), hand-computed timelines, the textbook
three-machine flow-shop recurrence, Johnson's rule, machine lower bounds, a
work-conservation upper bound, symmetry properties and brute force.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import cmodel
from oracle import model as M
from paper_1806_10113_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def rand_group(rng, n, lo=0, hi=60):
    return [tuple(int(v) for v in rng.integers(lo, hi, size=3)) for _ in range(n)]


# ------------------------------------------------------------------ P1 paper

def test_paper_worked_timeline():
    g = load("paper_worked_timeline.json")
    m = M.Model(**g["model"])
    T, ev = M.simulate(g["tasks_ns"], g["order"], m, trace=True)
    want = g["events_ns"]
    assert ev[("HtD", 0)] == want["HtD_0"]
    assert ev[("K", 0)] == want["K_0"]
    assert ev[("HtD", 1)] == want["HtD_1"]
    assert ev[("DtH", 0)] == want["DtH_0"]
    assert ev[("HtD", 2)] == want["HtD_2"]
    assert ev[("K", 1)][0] == want["K_1_start"]
    # the same instants come out of exact arithmetic (all are whole ns)
    Te, eve = M.simulate(g["tasks_ns"], g["order"], m, exact=True, trace=True)
    assert eve[("DtH", 0)][1] == Fraction(want["DtH_0"][1])
    assert eve[("HtD", 1)][1] == Fraction(want["HtD_1"][1])
    # and the C transcription gives the same total
    assert cmodel.simulate(g["tasks_ns"], g["order"], m) == T


def test_paper_timeline_without_slowdown_differs():
    # Without the overlap re-estimation HtD_1 would end at its solo time 210 ms,
    # which the text says is the value before re-estimation.
    g = load("paper_worked_timeline.json")
    _, ev = M.simulate(g["tasks_ns"], g["order"], M.Model(1, 1, 1), trace=True)
    assert ev[("HtD", 1)][1] == 210_000_000


# --------------------------------------------------------- hand computations

def test_hand_two_task():
    g = load("hand_two_task.json")
    for case in g["cases"]:
        m = M.Model(**case["model"])
        assert M.simulate(g["tasks_ns"], [0, 1], m) == case["T_01"]
        assert M.simulate(g["tasks_ns"], [1, 0], m) == case["T_10"]
        assert M.simulate(g["tasks_ns"], [1, 0], m, exact=True) == Fraction(case["exact_10"])
        assert cmodel.simulate(g["tasks_ns"], [0, 1], m) == case["T_01"]
        assert cmodel.simulate(g["tasks_ns"], [1, 0], m) == case["T_10"]


def test_bk100_no_slowdown():
    # BK100 = T0..T3 of the synthetic-task table; identity order by hand:
    # HtD ends 1,3,6,7 ms; K ends 9,16,22,29; DtH ends 10,17,23,31 -> 31 ms.
    bk = W.paper_benchmark("BK100")
    assert M.simulate(bk, [0, 1, 2, 3], M.NO_SLOWDOWN) == 31_000_000
    s = M.exhaustive(bk, M.NO_SLOWDOWN)
    # lower bound min h + sum k + min d = 1 + 28 + 1 = 30 ms is reached
    assert s["min_ns"] == 30_000_000


def test_dk_dt_classification():
    # Section 4.3: T0..T3 are dominant-kernel, T4..T7 dominant-transfer.
    for name, f in W.PAPER_TASKS_UNITS.items():
        t = [int(round(v * W.PAPER_UNIT_NS)) for v in f]
        assert M.dominant_kernel(t) == (name in ("T0", "T1", "T2", "T3"))


# ---------------------------------------------- P2 flow shop, P3 Johnson rule

def flow_shop(tasks, order):
    """Textbook three-machine permutation flow-shop completion times."""
    H = K = D = 0
    for x in order:
        h, k, d = tasks[x]
        H = H + h
        K = max(H, K) + k
        D = max(K, D) + d
    return D


def test_flow_shop_recurrence_at_full_speed():
    rng = np.random.default_rng(11)
    for _ in range(40):
        n = int(rng.integers(1, 6))
        tasks = rand_group(rng, n)
        for p in itertools.permutations(range(n)):
            assert M.simulate(tasks, p, M.NO_SLOWDOWN) == flow_shop(tasks, p)
    # a rate pair of q/q at any q is the same model
    tasks = rand_group(rng, 5)
    for p in itertools.permutations(range(5)):
        assert M.simulate(tasks, p, M.Model(8, 8, 8)) == flow_shop(tasks, p)


def johnson_makespan(a, b):
    first = sorted([i for i in range(len(a)) if a[i] <= b[i]], key=lambda i: a[i])
    last = sorted([i for i in range(len(a)) if a[i] > b[i]], key=lambda i: -b[i])
    t1 = t2 = 0
    for i in first + last:
        t1 += a[i]
        t2 = max(t1, t2) + b[i]
    return t2


def test_johnson_rule_two_machine_cases():
    rng = np.random.default_rng(12)
    for _ in range(25):
        n = int(rng.integers(2, 7))
        h = [int(v) for v in rng.integers(0, 40, n)]
        k = [int(v) for v in rng.integers(0, 40, n)]
        d = [int(v) for v in rng.integers(0, 40, n)]
        no_d = [(h[i], k[i], 0) for i in range(n)]
        assert M.exhaustive(no_d, M.NO_SLOWDOWN)["min_ns"] == johnson_makespan(h, k)
        no_h = [(0, k[i], d[i]) for i in range(n)]
        assert M.exhaustive(no_h, M.NO_SLOWDOWN)["min_ns"] == johnson_makespan(k, d)


# ------------------------------------------------------ P4, P5 bounds

MODELS = [M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN, M.Model(16, 9, 13), M.Model(2, 1, 1)]


def test_machine_lower_bounds():
    rng = np.random.default_rng(13)
    for _ in range(150):
        n = int(rng.integers(1, 7))
        tasks = rand_group(rng, n)
        h = [t[0] for t in tasks]; k = [t[1] for t in tasks]; d = [t[2] for t in tasks]
        for m in MODELS:
            p = list(rng.permutation(n))
            T = M.simulate(tasks, p, m)
            assert T >= sum(h) and T >= sum(k) and T >= sum(d)
            assert T >= sum(h) + min(k[i] + d[i] for i in range(n))
            assert T >= min(h) + sum(k) + min(d)
            assert T >= min(h[i] + k[i] for i in range(n)) + sum(d)


def test_serial_upper_bound_when_sharing_does_not_lose_bandwidth():
    rng = np.random.default_rng(14)
    for _ in range(150):
        n = int(rng.integers(1, 7))
        tasks = rand_group(rng, n)
        serial = sum(sum(t) for t in tasks)
        for m in (M.DEFAULT, M.NO_SLOWDOWN, M.Model(16, 9, 13), M.Model(2, 1, 1)):
            assert m.p_htd + m.p_dth >= m.q
            p = list(rng.permutation(n))
            assert M.simulate(tasks, p, m, exact=True) <= serial
            assert M.simulate(tasks, p, m) <= serial + 3 * n


def test_serial_bound_can_fail_at_paper_example_rates():
    # At 3/8 + 3/8 < 1, overlapping costs bandwidth: the two-task example
    # takes 14 ns against a serial sum of 14 ns in one order and the exact
    # model exceeds the serial sum for some groups.
    found = False
    rng = np.random.default_rng(15)
    for _ in range(200):
        tasks = rand_group(rng, 3, 1, 30)
        serial = sum(sum(t) for t in tasks)
        for p in itertools.permutations(range(3)):
            if M.simulate(tasks, p, M.PAPER_EXAMPLE, exact=True) > serial:
                found = True
    assert found


# ---------------------------------------------------------- P6, P7 invariants

def test_exhaustive_min_le_heuristic_and_mean_order():
    rng = np.random.default_rng(16)
    for _ in range(30):
        n = int(rng.integers(1, 7))
        tasks = rand_group(rng, n, 1, 50)
        for m in (M.DEFAULT, M.NO_SLOWDOWN):
            s = M.exhaustive(tasks, m)
            hp = M.heuristic(tasks, m)
            assert sorted(hp) == list(range(n))
            assert s["min_ns"] <= M.simulate(tasks, hp, m)
            assert s["min_ns"] <= s["mean_ns"] <= s["max_ns"]
            assert M.simulate(tasks, s["best"], m) == s["min_ns"]
            assert M.simulate(tasks, s["worst"], m) == s["max_ns"]


def test_single_task_and_identical_tasks():
    for m in MODELS:
        assert M.simulate([(5, 7, 11)], [0], m) == 23
        s = M.exhaustive([(3, 4, 5)] * 4, m)
        assert s["min_ns"] == s["max_ns"] == s["mean_ns"]


def test_relabeling_keeps_multiset():
    rng = np.random.default_rng(17)
    tasks = rand_group(rng, 5, 1, 40)
    perm = list(rng.permutation(5))
    relabeled = [tasks[i] for i in perm]
    for m in (M.DEFAULT, M.PAPER_EXAMPLE):
        a = sorted(M.all_times(tasks, m))
        b = sorted(M.all_times(relabeled, m))
        assert a == b


def test_zero_task_padding_at_tail():
    rng = np.random.default_rng(18)
    for _ in range(60):
        n = int(rng.integers(1, 6))
        tasks = rand_group(rng, n, 1, 40)
        p = list(rng.permutation(n))
        for m in MODELS:
            T = M.simulate(tasks, p, m)
            padded = tasks + [(0, 0, 0)] * 3
            assert M.simulate(padded, p + [n, n + 1, n + 2], m) == T


def test_zero_length_stages():
    # an empty transfer stage or kernel behaves like the command is absent
    tasks = [(0, 5, 3), (4, 0, 0), (2, 2, 0)]
    assert M.simulate(tasks, [0, 1, 2], M.NO_SLOWDOWN) == flow_shop(tasks, [0, 1, 2])
    for m in MODELS:
        for p in itertools.permutations(range(3)):
            assert M.simulate(tasks, p, m) == cmodel.simulate(tasks, p, m)


def test_flow_shop_reversibility():
    rng = np.random.default_rng(19)
    for _ in range(40):
        n = int(rng.integers(1, 7))
        tasks = rand_group(rng, n)
        p = list(rng.permutation(n))
        rev = [(d, k, h) for (h, k, d) in tasks]
        assert M.simulate(tasks, p, M.NO_SLOWDOWN) == M.simulate(rev, p[::-1], M.NO_SLOWDOWN)


# -------------------------------------------------------------- P8 rounding

def test_integer_mode_within_rounding_bound_of_exact():
    rng = np.random.default_rng(20)
    worst = 0
    for _ in range(300):
        n = int(rng.integers(1, 7))
        tasks = rand_group(rng, n, 0, 1000)
        for m in MODELS:
            p = list(rng.permutation(n))
            Ti = M.simulate(tasks, p, m)
            Te = M.simulate(tasks, p, m, exact=True)
            bound = 3 * n * math.ceil(m.q / min(m.p_htd, m.p_dth))
            worst = max(worst, abs(Ti - Te))
            assert abs(Ti - Te) <= bound
            if m.q == m.p_htd == m.p_dth:
                assert Ti == Te


# ---------------------------------------------------------- P10 enumeration

def test_rank_is_lexicographic_lehmer_index():
    for n in range(1, 7):
        for r, p in enumerate(itertools.permutations(range(n))):
            assert M.lehmer_rank(p) == r
            assert tuple(M.nth_permutation(n, r)) == p
    # the positional decode used above n = 8 agrees with itertools at n = 9
    it = itertools.permutations(range(9))
    for r, p in enumerate(itertools.islice(it, 0, 5000, 1)):
        if r % 997 == 0:
            assert M.lehmer_rank(p) == r


def test_summary_fields_by_brute_force():
    tasks = W.single_group_uniform(6, seed=3)
    s = M.exhaustive(tasks)
    times = s["times"]
    assert s["count"] == 720
    assert s["sum"] == sum(times)
    assert s["min_ns"] == min(times) and times.index(min(times)) == s["argmin_rank"]
    assert s["max_ns"] == max(times) and times.index(max(times)) == s["argmax_rank"]
    fp = sum((2 * r + 1) * t for r, t in enumerate(times)) % (1 << 64)
    assert s["fingerprint"] == fp


# ------------------------------------------------ C transcription == Python

def test_c_oracle_matches_python_oracle():
    rng = np.random.default_rng(21)
    for _ in range(60):
        n = int(rng.integers(1, 7))
        tasks = rand_group(rng, n, 0, 200)
        for m in MODELS + [M.Model(4, 3, 3, 1)]:
            s = M.exhaustive(tasks, m)
            c = cmodel.exhaustive(tasks, m, per_order=True, threads=3)
            assert list(c["times"]) == s["times"]
            for key in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "sum", "count", "fingerprint"):
                assert c[key] == s[key], key


def test_c_oracle_strided_and_ranged():
    tasks = W.single_group_uniform(7, seed=9)
    full = cmodel.exhaustive(tasks, per_order=True)
    times = full["times"]
    part = cmodel.exhaustive(tasks, lo=100, hi=3000, threads=4)
    assert part["sum"] == int(times[100:3000].sum())
    st = cmodel.exhaustive(tasks, lo=5, hi=5040, stride=7, threads=4)
    assert st["sum"] == int(times[5:5040:7].sum())
    assert st["count"] == len(range(5, 5040, 7))


# ------------------------------------------------------------- heuristic

def test_heuristic_hand_worked_cases():
    g = load("heuristic_hand.json")
    m = M.Model(**g["model"])
    for case in g["cases"]:
        order = M.heuristic(case["tasks"], m)
        assert order == case["order"], case["name"]
        if "T" in case:
            assert M.simulate(case["tasks"], order, m) == case["T"]


def test_heuristic_hand_worked_cases_overlapped_rates():
    """Hand-worked at 3/4: update under overlapped transfers, a select_next
    tie (lower index wins) and select_last, each intermediate update checked."""
    g = load("heuristic_hand_overlap.json")
    m = M.Model(**g["model"])
    for case in g["cases"]:
        tasks = case["tasks"]
        for key, want in case["updates"].items():
            ot = [int(v) for v in key.split(",")]
            assert list(M.update(tasks, ot, m)) == want, (case["name"], key)
        assert M.heuristic(tasks, m) == case["order"], case["name"]
        assert M.simulate(tasks, case["order"], m) == case["T"]
        assert cmodel.simulate(tasks, case["order"], m) == case["T"]


def test_heuristic_structure():
    rng = np.random.default_rng(22)
    for _ in range(50):
        n = int(rng.integers(1, 10))
        tasks = rand_group(rng, n, 1, 100)
        o = M.heuristic(tasks, M.DEFAULT)
        assert sorted(o) == list(range(n))
        # first task is the largest K - HtD (longer DtH, then lower index, on ties)
        key = [(-(t[1] - t[0]), -t[2], i) for i, t in enumerate(tasks)]
        assert o[0] == min(range(n), key=lambda i: key[i])


def test_heuristic_beats_average_on_paper_benchmarks_mostly():
    # The paper reports the heuristic below the average ordering on hardware;
    # under the model this is a statistic, not a law.  Record it for BK0..BK100.
    wins = 0
    for name in W.PAPER_BENCHMARKS:
        bk = W.paper_benchmark(name)
        s = M.exhaustive(bk, M.DEFAULT)
        T = M.simulate(bk, M.heuristic(bk, M.DEFAULT), M.DEFAULT)
        wins += T <= s["mean_ns"]
    assert wins >= 4


# ------------------------------------------------------ one DMA engine
# Section 3.2 (launch scheme for devices with one DMA engine): all HtDs go
# to the one transfer queue before any DtH; kernels use the other queue.

ONE_DMA = M.Model(4, 3, 3, 1)


def one_dma_recurrence(tasks, order):
    """Textbook recurrence for that scheme: the transfer engine is busy with
    the HtDs back to back until their sum, then serves the DtHs in order, each
    after its kernel; the kernel engine serves kernels in order, each after
    its HtD."""
    H = K = 0
    ks = []
    for x in order:
        h, k, _ = tasks[x]
        H += h
        K = max(H, K) + k
        ks.append(K)
    D = H
    for x, kend in zip(order, ks):
        D = max(D, kend) + tasks[x][2]
    return D


def test_one_dma_hand_worked_timelines():
    g = load("one_dma_hand.json")
    for case in g["cases"]:
        T, ev = M.simulate(case["tasks_ns"], case["order"], ONE_DMA, trace=True)
        assert T == case["T"]
        for name, (a, b) in case["events"].items():
            kind, x = name.split("_")
            assert ev[(kind, int(x))] == [a, b], name


def test_one_dma_closed_form_recurrence():
    rng = np.random.default_rng(31)
    for _ in range(60):
        n = int(rng.integers(1, 6))
        tasks = rand_group(rng, n, 0, 40)
        for p in itertools.permutations(range(n)):
            assert M.simulate(tasks, p, ONE_DMA) == one_dma_recurrence(tasks, p)


def test_one_dma_rates_do_not_matter():
    # one engine never moves data both ways at once, so no slowdown applies
    rng = np.random.default_rng(32)
    for _ in range(40):
        n = int(rng.integers(1, 6))
        tasks = rand_group(rng, n)
        p = list(rng.permutation(n))
        ts = {M.simulate(tasks, p, M.Model(q, ph, pd, 1), exact=ex)
              for q, ph, pd in ((4, 3, 3), (8, 3, 3), (1, 1, 1), (16, 9, 13)) for ex in (False, True)}
        assert len(ts) == 1


def test_one_dma_special_cases():
    rng = np.random.default_rng(33)
    for _ in range(25):
        n = int(rng.integers(2, 7))
        h = [int(v) for v in rng.integers(0, 40, n)]
        k = [int(v) for v in rng.integers(0, 40, n)]
        d = [int(v) for v in rng.integers(0, 40, n)]
        # no HtD work: two-machine flow shop (K, DtH), optimum by Johnson's rule
        no_h = [(0, k[i], d[i]) for i in range(n)]
        assert M.exhaustive(no_h, ONE_DMA)["min_ns"] == johnson_makespan(k, d)
        # no DtH work: two-machine flow shop (HtD, K)
        no_d = [(h[i], k[i], 0) for i in range(n)]
        assert M.exhaustive(no_d, ONE_DMA)["min_ns"] == johnson_makespan(h, k)
        # no kernel work: the transfer engine alone decides, for every ordering
        no_k = [(h[i], 0, d[i]) for i in range(n)]
        assert set(M.all_times(no_k, ONE_DMA)) == {sum(h) + sum(d)}


def test_one_dma_lower_bounds_and_serial_upper_bound():
    rng = np.random.default_rng(34)
    for _ in range(150):
        n = int(rng.integers(1, 7))
        tasks = rand_group(rng, n)
        h = [t[0] for t in tasks]; k = [t[1] for t in tasks]; d = [t[2] for t in tasks]
        p = list(rng.permutation(n))
        T = M.simulate(tasks, p, ONE_DMA)
        assert sum(h) + sum(d) <= T <= sum(h) + sum(k) + sum(d)
        assert T >= min(h) + sum(k) + min(d)
        # one engine is never faster than two at full speed
        assert T >= M.simulate(tasks, p, M.NO_SLOWDOWN)


def test_one_dma_heuristic_is_a_valid_ordering():
    for seed in range(6):
        tasks = W.single_group_uniform(7, seed)
        h = M.heuristic(tasks, ONE_DMA)
        assert sorted(h) == list(range(7))
        assert M.exhaustive(tasks, ONE_DMA)["min_ns"] <= M.simulate(tasks, h, ONE_DMA)
