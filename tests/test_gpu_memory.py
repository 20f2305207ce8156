"""GPU parity of the device-memory-limit evaluator (task buffers held from
HtD start to DtH end, at most a capacity at once): every ordering, the
summary and Algorithm 1 under the limit against the CPU oracle, bit for bit."""
import math

import numpy as np
import pytest

from oracle import cmodel
from oracle import memory as MM
from oracle import model as M
from paper_1806_10113_amd import workloads as W

pytestmark = pytest.mark.gpu

MODELS = [M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN, M.Model(16, 9, 13), M.Model(4, 3, 3, 1)]


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_10113_amd import tgo
    tgo.lib()
    return torch.device("cuda:0")


def to_dev(a, dev, dtype=np.int64):
    import torch
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=dtype))).to(dev)


def tmodel(m: M.Model):
    from paper_1806_10113_amd import tgo
    return tgo.Model(int(math.log2(m.q)), m.p_htd, m.p_dth, m.dma_engines)


def run(dev, tasks, mem, cap, m, per_order=True):
    from paper_1806_10113_amd import tgo
    s, po = tgo.exhaustive_mem(to_dev(tasks, dev), to_dev(mem, dev), cap, tmodel(m), per_order=per_order)
    return tgo.read_summary(s), (po.cpu().numpy() if po is not None else None)


def check_summary(s, times, n):
    # the summary rules (lowest rank on ties; fingerprint = sum of (2r+1) T
    # mod 2^64), applied with numpy so that 11! and 12! orderings stay cheap
    t = np.asarray(times, dtype=np.int64)
    assert len(t) == math.factorial(n)
    assert s["status"] == 0 and s["n"] == n and s["count"] == len(t)
    lo, hi = int(np.argmin(t)), int(np.argmax(t))
    assert (s["min_ns"], s["argmin_rank"]) == (int(t[lo]), lo)
    assert (s["max_ns"], s["argmax_rank"]) == (int(t[hi]), hi)
    total = int(t.sum(dtype=np.int64))
    assert s["sum"] == total
    r = np.arange(len(t), dtype=np.uint64)
    assert s["fingerprint"] == int(((2 * r + 1) * t.astype(np.uint64)).sum(dtype=np.uint64))
    assert s["best"] == list(M.nth_permutation(n, lo)) and s["worst"] == list(M.nth_permutation(n, hi))
    assert abs(s["mean_ns"] - total / len(t)) <= 1e-12 * max(1.0, total / len(t))


def check_heuristic(s, tasks, mem, cap, m):
    h = MM.heuristic([tuple(int(v) for v in t) for t in tasks], mem, cap, m)
    assert s["heur"] == h
    assert s["heur_ns"] == MM.simulate(tasks, mem, cap, h, m)


def test_small_groups_every_ordering(dev):
    rng = np.random.default_rng(70)
    for trial in range(12):
        n = int(rng.integers(1, 7))
        tasks = rng.integers(0, 3000, size=(n, 3))
        mem = rng.integers(0, 100, size=n)
        caps = sorted({max(1, int(mem.max())), int(mem.sum()) // 2 + 1, max(1, int(mem.sum()))})
        for cap in caps:
            cap = max(cap, int(mem.max()), 1)
            for m in MODELS:
                s, po = run(dev, tasks, mem, cap, m)
                want = MM.all_times(tasks.tolist(), mem.tolist(), cap, m)
                assert list(po) == want, (trial, n, cap, m)
                check_summary(s, want, n)
                check_heuristic(s, tasks.tolist(), mem.tolist(), cap, m)


def test_n8_capacities_against_oracle(dev):
    # 40,320 orderings: 158 blocks of 256 lanes, the last one half full
    tasks = W.single_group_uniform(8, seed=0)
    mem = W.footprints(tasks)
    for frac in (0.0, 0.2, 0.35, 0.5, 0.75, 1.0):
        cap = W.capacity_fraction(mem, frac)
        for m in (M.DEFAULT, M.PAPER_EXAMPLE, M.Model(4, 3, 3, 1)):
            s, po = run(dev, tasks, mem, cap, m)
            want = cmodel.mem_times(tasks, mem, cap, m)
            assert np.array_equal(po, want), (frac, m)
            check_summary(s, want, 8)
            check_heuristic(s, tasks.tolist(), mem.tolist(), cap, m)


def test_enough_memory_equals_unconstrained_search(dev):
    from paper_1806_10113_amd import tgo
    tasks = W.single_group_uniform(8, seed=0)
    mem = W.footprints(tasks)
    for m in (M.DEFAULT, M.Model(4, 3, 3, 1)):
        s, po = run(dev, tasks, mem, int(mem.sum()), m)
        e, epo = tgo.exhaustive(to_dev(tasks, dev), tmodel(m), per_order=True)
        e = tgo.read_summary(e)
        assert np.array_equal(po, epo.cpu().numpy())
        for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "sum", "fingerprint", "best", "worst"):
            assert s[k] == e[k]
        assert s["heur"] == M.heuristic(tasks.tolist(), m)


def test_serial_capacity_is_serial_sum(dev):
    # footprints above half the capacity: one task resident at a time
    rng = np.random.default_rng(71)
    tasks = rng.integers(0, 10 ** 6, size=(7, 3))
    mem = rng.integers(501, 1001, size=7)
    for m in (M.DEFAULT, M.Model(4, 3, 3, 1)):
        s, po = run(dev, tasks, mem, 1000, m)
        assert (po == int(tasks.sum())).all()
        assert s["min_ns"] == s["max_ns"] == s["heur_ns"] == int(tasks.sum())


def test_n11_summary_against_c_oracle(dev):
    # 39,916,800 orderings, summary only, compared with the C transcription
    tasks = W.single_group_mixed(12, seed=1)[:11]
    mem = W.footprints(tasks)
    for frac, m in ((0.3, M.DEFAULT), (0.5, M.Model(4, 3, 3, 1))):
        cap = W.capacity_fraction(mem, frac)
        s, _ = run(dev, tasks, mem, cap, m, per_order=False)
        check_summary(s, cmodel.mem_times(tasks, mem, cap, m), 11)
        check_heuristic(s, tasks.tolist(), mem.tolist(), cap, m)


def test_n12_full_size_sampled(dev):
    # the N = 12 group at its full 12! orderings: the reported extremes are
    # checked by the oracle, and the per-ordering output on sampled ranks
    from paper_1806_10113_amd import tgo
    tasks = W.single_group_mixed(12, seed=1)
    mem = W.footprints(tasks)
    cap = W.capacity_fraction(mem, 0.4)
    m = M.DEFAULT
    s, po = run(dev, tasks, mem, cap, m)
    assert s["status"] == 0 and s["count"] == math.factorial(12)
    assert MM.simulate(tasks, mem, cap, s["best"], m) == s["min_ns"]
    assert MM.simulate(tasks, mem, cap, s["worst"], m) == s["max_ns"]
    assert M.lehmer_rank(s["best"]) == s["argmin_rank"] and M.lehmer_rank(s["worst"]) == s["argmax_rank"]
    assert int(po.min()) == s["min_ns"] and int(po.max()) == s["max_ns"]
    assert int(np.argmin(po)) == s["argmin_rank"] and int(np.argmax(po)) == s["argmax_rank"]
    assert int(po.sum(dtype=np.int64)) == s["sum"]
    rng = np.random.default_rng(72)
    ranks = rng.integers(0, math.factorial(12), size=300)
    for r in ranks:
        p = M.nth_permutation(12, int(r))
        assert po[r] == cmodel.mem_simulate(tasks, mem, cap, p, m)
    check_heuristic(s, tasks.tolist(), mem.tolist(), cap, m)
    # evaluate_mem on the same sampled orderings
    orders = np.array([M.nth_permutation(12, int(r)) for r in ranks], dtype=np.uint8)
    got = tgo.evaluate_mem(to_dev(tasks, dev), to_dev(mem, dev), cap, to_dev(orders, dev, np.uint8),
                           tmodel(m)).cpu().numpy()
    assert np.array_equal(got, po[ranks])


def test_evaluate_mem_rows(dev):
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(73)
    for n in (1, 5, 13, 16):
        tasks = rng.integers(0, 10 ** 6, size=(n, 3))
        mem = rng.integers(0, 10 ** 4, size=n)
        cap = W.capacity_fraction(mem, 0.3)
        orders = np.array([rng.permutation(n) for _ in range(777)], dtype=np.uint8)
        orders[5] = 0                                   # not a permutation (n > 1)
        for m in (M.DEFAULT, M.Model(4, 3, 3, 1)):
            got = tgo.evaluate_mem(to_dev(tasks, dev), to_dev(mem, dev), cap, to_dev(orders, dev, np.uint8),
                                   tmodel(m)).cpu().numpy()
            for i in range(len(orders)):
                if n > 1 and i == 5:
                    assert got[i] == tgo.TGO_EINVAL
                else:
                    assert got[i] == cmodel.mem_simulate(tasks, mem, cap, orders[i], m)


def test_edge_cases(dev):
    from paper_1806_10113_amd import tgo
    # one task; zero durations; zero footprints; a footprint equal to the capacity
    s, po = run(dev, [[5, 7, 11]], [9], 9, M.DEFAULT)
    assert list(po) == [23] and s["heur"] == [0] and s["heur_ns"] == 23
    tasks = [[0, 0, 0], [3, 0, 4], [0, 5, 0], [2, 2, 2]]
    for mem, cap in (([0, 0, 0, 0], 1), ([4, 0, 4, 3], 4), ([4, 4, 4, 4], 7)):
        for m in MODELS:
            s, po = run(dev, tasks, mem, cap, m)
            assert list(po) == MM.all_times(tasks, mem, cap, m)
            check_heuristic(s, tasks, mem, cap, m)
    # a task that cannot fit, a negative footprint, durations out of range
    for mem, cap, tk, code in (([3, 11], 10, [[1, 1, 1], [1, 1, 1]], tgo.TGO_EINVAL),
                               ([3, -1], 10, [[1, 1, 1], [1, 1, 1]], tgo.TGO_EINVAL),
                               ([3, 3], 10, [[1, 1, 1], [1 << 41, 1, 1]], tgo.TGO_ERANGE)):
        s, _ = run(dev, tk, mem, cap, M.DEFAULT, per_order=False)
        assert s["status"] == code and s["heur_ns"] == code
        got = tgo.evaluate_mem(to_dev(tk, dev), to_dev(mem, dev), cap,
                               to_dev([[0, 1], [1, 0]], dev, np.uint8)).cpu().numpy()
        assert (got == code).all()


def _stored():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "memory_n12_summaries.json")))


@pytest.mark.parametrize("case", ["dma2_cap1", "dma2_cap0.6", "dma2_cap0.4", "dma2_cap0.25", "dma2_cap0",
                                  "dma1_cap1", "dma1_cap0.6", "dma1_cap0.4", "dma1_cap0.25", "dma1_cap0"])
def test_n12_full_size_against_stored_oracle(dev, case):
    """The N = 12 group under the memory limit at five capacities and both
    launch schemes: every field of the summary over all 12! orderings, and
    Algorithm 1 under the limit, equal the oracle's stored values
    (tests/golden/memory_n12_summaries.json, written by make_golden.py from
    the oracle alone)."""
    g = _stored()
    c = g["cases"][case]
    tasks = np.array(g["tasks_ns"], dtype=np.int64)
    mem = np.array(g["mem_bytes"], dtype=np.int64)
    assert np.array_equal(tasks, W.single_group_mixed(12, seed=1))
    assert np.array_equal(mem, W.footprints(tasks))
    m = M.Model(**c["model"])
    s, _ = run(dev, tasks, mem, c["capacity"], m, per_order=False)
    assert s["status"] == 0 and s["count"] == c["count"]
    for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank"):
        assert s[k] == c[k], k
    assert s["sum"] == int(c["sum"]) and s["fingerprint"] == int(c["fingerprint"])
    assert s["heur"] == c["heuristic"] and s["heur_ns"] == c["heuristic_ns"]
