"""GPU parity: the HIP kernels, called through the C ABI, against the CPU
oracle on the same seeded inputs.  Integer results must agree bit for bit."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import cmodel
from oracle import model as M
from paper_1806_10113_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_10113_amd import tgo
    tgo.lib()  # fail loudly if the HIP library is missing
    return torch.device("cuda:0")


def to_dev(a, dev, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(dev)


def tmodel(m: M.Model):
    from paper_1806_10113_amd import tgo
    return tgo.Model(int(math.log2(m.q)), m.p_htd, m.p_dth, m.dma_engines)


MODELS = [M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN, M.Model(16, 9, 13), M.Model(4, 1, 4),
          M.Model(1024, 1000, 3)]


def rand_tasks(rng, n, hi):
    return rng.integers(0, hi, size=(n, 3)).astype(np.int64)


# ------------------------------------------------------------------ evaluate

def test_evaluate_random_orderings(dev):
    import torch
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(100)
    for n in list(range(1, 17)):
        for hi in (4, 1000, 20_000_000):
            tasks = rand_tasks(rng, n, hi)
            orders = np.stack([rng.permutation(n) for _ in range(700)]).astype(np.uint8)
            for m in MODELS:
                want = cmodel.eval_orders(tasks, orders, m)
                got = tgo.evaluate(to_dev(tasks, dev), to_dev(orders, dev), tmodel(m))
                torch.cuda.synchronize()
                assert np.array_equal(got.cpu().numpy(), want), (n, hi, m)


def test_evaluate_64bit_time_path(dev):
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(101)
    for n in (3, 9, 16):
        # durations near 2^39 ns force the 64-bit path
        tasks = rng.integers(1 << 30, 1 << 39, size=(n, 3)).astype(np.int64)
        orders = np.stack([rng.permutation(n) for _ in range(300)]).astype(np.uint8)
        for m in (M.DEFAULT, M.Model(1024, 7, 1000)):
            want = cmodel.eval_orders(tasks, orders, m)
            got = tgo.evaluate(to_dev(tasks, dev), to_dev(orders, dev), tmodel(m)).cpu().numpy()
            assert np.array_equal(got, want)


def test_evaluate_paper_timeline_and_hand_cases(dev):
    from paper_1806_10113_amd import tgo
    g = json.load(open(os.path.join(GOLDEN, "paper_worked_timeline.json")))
    tasks = np.array(g["tasks_ns"], dtype=np.int64)
    orders = np.array([[0, 1, 2]], dtype=np.uint8)
    got = tgo.evaluate(to_dev(tasks, dev), to_dev(orders, dev), tgo.PAPER_EXAMPLE).cpu().numpy()
    assert got[0] == M.simulate(tasks, [0, 1, 2], M.PAPER_EXAMPLE)
    h = json.load(open(os.path.join(GOLDEN, "hand_two_task.json")))
    tasks = np.array(h["tasks_ns"], dtype=np.int64)
    orders = np.array([[0, 1], [1, 0]], dtype=np.uint8)
    for case in h["cases"]:
        mm = case["model"]
        m = tgo.Model(int(math.log2(mm["q"])), mm["p_htd"], mm["p_dth"])
        got = tgo.evaluate(to_dev(tasks, dev), to_dev(orders, dev), m).cpu().numpy()
        assert list(got) == [case["T_01"], case["T_10"]]


def test_evaluate_errors_on_device_data(dev):
    from paper_1806_10113_amd import tgo
    tasks = np.array([[1, 2, 3], [4, 5, 6], [7, 8, 9]], dtype=np.int64)
    orders = np.array([[0, 1, 2], [0, 0, 1], [2, 1, 3], [2, 1, 0]], dtype=np.uint8)
    got = tgo.evaluate(to_dev(tasks, dev), to_dev(orders, dev)).cpu().numpy()
    assert got[0] == M.simulate(tasks, [0, 1, 2]) and got[3] == M.simulate(tasks, [2, 1, 0])
    assert got[1] == tgo.TGO_EINVAL and got[2] == tgo.TGO_EINVAL
    bad = tasks.copy()
    bad[1, 2] = -5
    got = tgo.evaluate(to_dev(bad, dev), to_dev(orders, dev)).cpu().numpy()
    assert (got == tgo.TGO_ERANGE).all()
    big = tasks.copy()
    big[0, 0] = 1 << 40
    got = tgo.evaluate(to_dev(big, dev), to_dev(orders, dev)).cpu().numpy()
    assert (got == tgo.TGO_ERANGE).all()


# ---------------------------------------------------------------- exhaustive

def check_summary(s, ref, n):
    assert s["status"] == 0
    assert s["count"] == math.factorial(n)
    for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "fingerprint"):
        assert int(s[k]) == int(ref[k]), k
    assert s["sum"] == int(ref["sum"])
    assert abs(s["mean_ns"] - float(ref["mean_ns"])) <= 2e-16 * abs(float(ref["mean_ns"]))
    assert s["best"] == list(M.nth_permutation(n, int(ref["argmin_rank"])))
    assert s["worst"] == list(M.nth_permutation(n, int(ref["argmax_rank"])))


def test_exhaustive_small_groups_per_ordering(dev):
    import torch
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(102)
    for n in range(1, 10):
        for hi in (3, 50_000, 20_000_000):
            tasks = rand_tasks(rng, n, hi)
            for m in (M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN, M.Model(16, 9, 13)):
                ref = cmodel.exhaustive(tasks, m, per_order=True)
                summ, po = tgo.exhaustive(to_dev(tasks, dev), tmodel(m), per_order=True)
                torch.cuda.synchronize()
                assert np.array_equal(po.cpu().numpy(), ref["times"]), (n, hi, m)
                check_summary(tgo.read_summary(summ), ref, n)


def test_exhaustive_ties_lowest_rank(dev):
    from paper_1806_10113_amd import tgo
    # identical tasks: every ordering ties, argmin = argmax = rank 0
    tasks = np.array([[5, 7, 3]] * 7, dtype=np.int64)
    s = tgo.read_summary(tgo.exhaustive(to_dev(tasks, dev))[0])
    assert s["argmin_rank"] == 0 and s["argmax_rank"] == 0 and s["min_ns"] == s["max_ns"]
    # all zero durations
    z = np.zeros((6, 3), dtype=np.int64)
    s = tgo.read_summary(tgo.exhaustive(to_dev(z, dev))[0])
    assert s["min_ns"] == 0 and s["max_ns"] == 0 and s["argmax_rank"] == 0 and s["sum"] == 0


def test_exhaustive_n10_per_ordering(dev):
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(4, 10, 10, seed=7)
    for g in range(b.n_groups):
        tasks = b.group(g)
        ref = cmodel.exhaustive(tasks, M.DEFAULT, per_order=True)
        summ, po = tgo.exhaustive(to_dev(tasks, dev), per_order=True)
        assert np.array_equal(po.cpu().numpy(), ref["times"])
        check_summary(tgo.read_summary(summ), ref, 10)


def test_exhaustive_grid_sizes_agree(dev, monkeypatch):
    """The launch grid does not change the answer: one block (each lane strides
    over hundreds of subtrees, folding them in rank order), a few blocks, and
    the default grid of many short blocks; ties are resolved to the lowest
    rank across block partials.  TGO_EXHAUSTIVE_BLOCKS sets the grid."""
    from paper_1806_10113_amd import tgo
    tasks = W.batch_groups(2, 9, 9, seed=11).group(0)
    ties = np.array([[5, 7, 3]] * 8, dtype=np.int64)
    models = (M.DEFAULT, M.Model(4, 3, 3, 1))
    refs = {m: cmodel.exhaustive(tasks, m, per_order=True) for m in models}
    for blocks in (None, "1", "3", "200"):
        if blocks is None:
            monkeypatch.delenv("TGO_EXHAUSTIVE_BLOCKS", raising=False)
        else:
            monkeypatch.setenv("TGO_EXHAUSTIVE_BLOCKS", blocks)
        for m in models:
            summ, po = tgo.exhaustive(to_dev(tasks, dev), tmodel(m), per_order=True)
            assert np.array_equal(po.cpu().numpy(), refs[m]["times"]), (blocks, m)
            check_summary(tgo.read_summary(summ), refs[m], 9)
            s = tgo.read_summary(tgo.exhaustive(to_dev(ties, dev), tmodel(m))[0])
            assert s["argmin_rank"] == 0 and s["argmax_rank"] == 0 and s["min_ns"] == s["max_ns"], (blocks, m)
    monkeypatch.delenv("TGO_EXHAUSTIVE_BLOCKS", raising=False)


def test_exhaustive_ties_across_subtrees(dev, monkeypatch):
    """Lanes meet their subtrees out of rank order (set-major), so equal
    times in different subtrees must still resolve to the lowest rank: groups
    whose tasks come in identical pairs (every ordering ties with the ones
    that swap equal tasks) against the oracle, on one block (each lane folds
    hundreds of subtrees), a few blocks and the default grid."""
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(21)
    groups = []
    for n in (8, 9, 10):
        base = rng.integers(1, 40, size=((n + 1) // 2, 3))
        groups.append(np.concatenate([base, base])[:n][rng.permutation(n)].astype(np.int64))
    models = (M.DEFAULT, M.Model(4, 3, 3, 1))
    refs = {(i, m): cmodel.exhaustive(g, m) for i, g in enumerate(groups) for m in models}
    for blocks in (None, "1", "3"):
        if blocks is None:
            monkeypatch.delenv("TGO_EXHAUSTIVE_BLOCKS", raising=False)
        else:
            monkeypatch.setenv("TGO_EXHAUSTIVE_BLOCKS", blocks)
        for i, g in enumerate(groups):
            for m in models:
                s = tgo.read_summary(tgo.exhaustive(to_dev(g, dev), tmodel(m))[0])
                check_summary(s, refs[(i, m)], len(g))
    monkeypatch.delenv("TGO_EXHAUSTIVE_BLOCKS", raising=False)


def test_exhaustive_concurrent_streams(dev):
    """Calls in flight on two streams at once do not share scratch memory:
    each gets the oracle's per-ordering times and summary (two groups, both
    DMA schemes, several calls queued per stream before any sync)."""
    import torch
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(2, 9, 9, seed=13)
    ga, gb = b.group(0), b.group(1)
    refs = {(k, m): cmodel.exhaustive(g, m, per_order=True)
            for k, g in (("a", ga), ("b", gb)) for m in (M.DEFAULT, M.Model(4, 3, 3, 1))}
    sa, sb = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    ta, tb = to_dev(ga, dev), to_dev(gb, dev)
    torch.cuda.synchronize()
    outs = []
    for m in (M.DEFAULT, M.Model(4, 3, 3, 1)):
        for _ in range(3):
            with torch.cuda.stream(sa):
                outs.append(("a", m, tgo.exhaustive(ta, tmodel(m), per_order=True, stream=sa)))
            with torch.cuda.stream(sb):
                outs.append(("b", m, tgo.exhaustive(tb, tmodel(m), per_order=True, stream=sb)))
    torch.cuda.synchronize()
    for k, m, (summ, po) in outs:
        ref = refs[(k, m)]
        assert np.array_equal(po.cpu().numpy(), ref["times"]), (k, m)
        check_summary(tgo.read_summary(summ), ref, 9)


def test_exhaustive_64bit_path(dev):
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(103)
    for n in (4, 8):
        tasks = rng.integers(1 << 33, 1 << 39, size=(n, 3)).astype(np.int64)
        ref = cmodel.exhaustive(tasks, M.DEFAULT, per_order=True)
        summ, po = tgo.exhaustive(to_dev(tasks, dev), per_order=True)
        assert np.array_equal(po.cpu().numpy(), ref["times"])
        check_summary(tgo.read_summary(summ), ref, n)


def test_exhaustive_device_errors(dev):
    from paper_1806_10113_amd import tgo
    tasks = np.array([[1, 2, 3], [4, -5, 6], [7, 8, 9]], dtype=np.int64)
    s = tgo.read_summary(tgo.exhaustive(to_dev(tasks, dev))[0])
    assert s["status"] == tgo.TGO_ERANGE


def test_exhaustive_uniform_n8_golden(dev):
    """Single group, N=8, log-uniform [10 us, 10 ms], seed 0: every ordering."""
    from paper_1806_10113_amd import tgo
    gold = json.load(open(os.path.join(GOLDEN, "single_group_summaries.json")))
    for key, m in (("uniform_n8_seed0", M.DEFAULT), ("uniform_n8_seed0_paper_rates", M.PAPER_EXAMPLE)):
        g = gold[key]
        tasks = W.single_group_uniform(8, 0)
        assert tasks.tolist() == g["tasks_ns"]
        ref = cmodel.exhaustive(tasks, m, per_order=True)
        summ, po = tgo.exhaustive(to_dev(tasks, dev), tmodel(m), per_order=True)
        assert np.array_equal(po.cpu().numpy(), ref["times"])
        check_summary(tgo.read_summary(summ), g, 8)


def test_exhaustive_mixed_n12_golden(dev):
    """Single group, N=12 (6 DK + 6 DT), seed 1: all 479,001,600 orderings in one
    call against the oracle's stored full enumeration, plus sampled ranks."""
    import torch
    from paper_1806_10113_amd import tgo
    g = json.load(open(os.path.join(GOLDEN, "single_group_summaries.json")))["mixed_n12_seed1"]
    tasks = W.single_group_mixed(12, 1)
    assert tasks.tolist() == g["tasks_ns"]
    summ, _ = tgo.exhaustive(to_dev(tasks, dev))
    s = tgo.read_summary(summ)
    check_summary(s, g, 12)
    # sampled orderings, evaluated one by one by the oracle and by the kernel
    rng = np.random.default_rng(104)
    ranks = rng.integers(0, math.factorial(12), size=2000)
    orders = np.array([M.nth_permutation(12, int(r)) for r in ranks], dtype=np.uint8)
    got = tgo.evaluate(to_dev(tasks, dev), to_dev(orders, dev)).cpu().numpy()
    want = cmodel.eval_orders(tasks, orders, M.DEFAULT)
    assert np.array_equal(got, want)
    assert (got >= s["min_ns"]).all() and (got <= s["max_ns"]).all()


# ----------------------------------------------------------------- heuristic

def test_heuristic_batch_against_oracle(dev):
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(300, 1, 16, seed=105)
    for m in (M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN):
        orders, ns = tgo.heuristic(to_dev(b.tasks, dev), to_dev(b.offs, dev), tmodel(m))
        orders = orders.cpu().numpy()
        ns = ns.cpu().numpy()
        for gi in range(b.n_groups):
            tasks = b.group(gi)
            n = len(tasks)
            want = M.heuristic(tasks, m)
            assert list(orders[gi, :n]) == want, gi
            assert (orders[gi, n:] == 0xFF).all()
            assert ns[gi] == M.simulate(tasks, want, m)


def test_heuristic_hand_cases_and_paper_benchmarks(dev):
    from paper_1806_10113_amd import tgo
    h = json.load(open(os.path.join(GOLDEN, "heuristic_hand.json")))
    groups = [np.array(c["tasks"], dtype=np.int64) for c in h["cases"]]
    groups += [W.paper_benchmark(k) for k in W.PAPER_BENCHMARKS]
    tasks = np.concatenate(groups)
    offs = np.cumsum([0] + [len(g) for g in groups]).astype(np.int32)
    orders, ns = tgo.heuristic(to_dev(tasks, dev), to_dev(offs, dev), tgo.NO_SLOWDOWN)
    orders = orders.cpu().numpy()
    for i, c in enumerate(h["cases"]):
        assert list(orders[i, :len(c["order"])]) == c["order"]
    for i, g in enumerate(groups):
        assert list(orders[i, :len(g)]) == M.heuristic(g, M.NO_SLOWDOWN)


def johnson_makespan(a, b):
    """Johnson's rule for the two-machine flow shop (a first, then b)."""
    first = sorted([i for i in range(len(a)) if a[i] <= b[i]], key=lambda i: a[i])
    last = sorted([i for i in range(len(a)) if a[i] > b[i]], key=lambda i: -b[i])
    t1 = t2 = 0
    for i in first + last:
        t1 += a[i]
        t2 = max(t1, t2) + b[i]
    return t2


def test_exhaustive_n13_largest_group(dev):
    """N = 13, the largest group enumerated (6,227,020,800 orderings, ranks
    beyond 32 bits), checked through closed forms that hold at any size."""
    from paper_1806_10113_amd import tgo
    n, R = 13, math.factorial(13)
    rng = np.random.default_rng(106)
    # identical tasks: every ordering ties
    same = np.array([[300_000, 900_000, 200_000]] * n, dtype=np.int64)
    s = tgo.read_summary(tgo.exhaustive(to_dev(same, dev))[0])
    T = M.simulate(same, list(range(n)), M.DEFAULT)
    assert s["status"] == 0 and s["count"] == R
    assert s["min_ns"] == T and s["max_ns"] == T and s["argmin_rank"] == 0 and s["argmax_rank"] == 0
    assert s["sum"] == T * R and s["fingerprint"] == (T * R * R) % (1 << 64)
    # full-speed transfers and no HtD work: Johnson's two-machine flow shop
    t = rng.integers(0, 2_000_000, size=(n, 3)).astype(np.int64)
    t[:, 0] = 0
    s = tgo.read_summary(tgo.exhaustive(to_dev(t, dev), tmodel(M.NO_SLOWDOWN))[0])
    assert s["min_ns"] == johnson_makespan(t[:, 1].tolist(), t[:, 2].tolist())
    # a general group under the default model: the reported extremes are
    # reproduced by their orderings, and sampled orderings lie between them
    t = W.single_group_mixed(n, 7)
    s = tgo.read_summary(tgo.exhaustive(to_dev(t, dev))[0])
    assert s["status"] == 0 and s["count"] == R
    assert cmodel.simulate(t, s["best"], M.DEFAULT) == s["min_ns"]
    assert cmodel.simulate(t, s["worst"], M.DEFAULT) == s["max_ns"]
    assert s["argmin_rank"] == M.lehmer_rank(s["best"]) and s["argmax_rank"] == M.lehmer_rank(s["worst"])
    assert s["min_ns"] <= s["mean_ns"] <= s["max_ns"]
    ranks = rng.integers(0, R, size=3000)
    orders = np.array([M.nth_permutation(n, int(r)) for r in ranks], dtype=np.uint8)
    got = tgo.evaluate(to_dev(t, dev), to_dev(orders, dev)).cpu().numpy()
    assert np.array_equal(got, cmodel.eval_orders(t, orders, M.DEFAULT))
    assert (got >= s["min_ns"]).all() and (got <= s["max_ns"]).all()


@pytest.mark.parametrize("key,dma", [("mixed_n13_seed7", 2), ("mixed_n13_seed1_one_dma", 1)])
def test_exhaustive_n13_against_stored_oracle(dev, key, dma):
    """The general N = 13 groups (6 DK + 7 DT, seeds 7 and 1): all
    6,227,020,800 orderings in one call, every summary field against the
    oracle's stored full enumeration (tests/golden/make_golden.py), and
    Algorithm 1's ordering and time."""
    from paper_1806_10113_amd import tgo
    g = json.load(open(os.path.join(GOLDEN, "single_group_summaries.json")))[key]
    seed = 7 if dma == 2 else 1
    tasks = W.single_group_mixed(13, seed)
    assert tasks.tolist() == g["tasks_ns"]
    m = M.Model(g["model"]["q"], g["model"]["p_htd"], g["model"]["p_dth"], g["model"]["dma_engines"])
    assert m.dma_engines == dma
    s = tgo.read_summary(tgo.exhaustive(to_dev(tasks, dev), tmodel(m))[0])
    check_summary(s, g, 13)
    orders, ns = tgo.heuristic(to_dev(tasks, dev), to_dev(np.array([0, 13], dtype=np.int32), dev), tmodel(m))
    assert list(orders.cpu().numpy()[0, :13]) == g["heuristic"]
    assert int(ns.cpu().numpy()[0]) == g["heuristic_ns"]


def test_predict_host_buffers(dev):
    """tgo_predict: one ordering from host memory, computed on the device."""
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(107)
    for n in (1, 2, 5, 9, 16):
        tasks = rand_tasks(rng, n, 20_000_000)
        for m in (M.DEFAULT, M.PAPER_EXAMPLE, M.Model(4, 3, 3, 1)):
            order = [int(v) for v in rng.permutation(n)]
            assert tgo.predict(tasks, order, tmodel(m)) == M.simulate(tasks, order, m)
    g = json.load(open(os.path.join(GOLDEN, "paper_worked_timeline.json")))
    m = M.Model(**g["model"])
    assert tgo.predict(np.array(g["tasks_ns"]), g["order"], tmodel(m)) == M.simulate(g["tasks_ns"], g["order"], m)
    with pytest.raises(tgo.TgoError):
        tgo.predict(rand_tasks(rng, 3, 100), [0, 0, 1])
    with pytest.raises(tgo.TgoError):
        tgo.predict(np.array([[1, -2, 3], [4, 5, 6]]), [0, 1])
