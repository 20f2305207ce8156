"""GPU parity for a device with one DMA engine (Section 3.2, launch scheme
with two command queues: every HtD before every DtH on the one transfer
queue).  Every entry point takes the scheme through tgo_model.dma_engines;
integer results must agree with the CPU oracle bit for bit."""
import json
import math
import os

import numpy as np
import pytest

from oracle import cmodel
from oracle import model as M
from oracle import philox
from paper_1806_10113_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ONE = M.Model(4, 3, 3, 1)
ONE_MODELS = [ONE, M.Model(8, 3, 3, 1), M.Model(1, 1, 1, 1), M.Model(1024, 1000, 3, 1)]
MASK64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_10113_amd import tgo
    tgo.lib()
    return torch.device("cuda:0")


def to_dev(a, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(dev)


def tmodel(m: M.Model):
    from paper_1806_10113_amd import tgo
    return tgo.Model(int(math.log2(m.q)), m.p_htd, m.p_dth, m.dma_engines)


def check_summary(s, ref, n):
    assert s["status"] == 0
    assert s["count"] == math.factorial(n)
    for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "fingerprint"):
        assert int(s[k]) == int(ref[k]), k
    assert s["sum"] == int(ref["sum"])
    assert abs(s["mean_ns"] - float(ref["mean_ns"])) <= 2e-16 * abs(float(ref["mean_ns"]))
    assert s["best"] == list(M.nth_permutation(n, int(ref["argmin_rank"])))
    assert s["worst"] == list(M.nth_permutation(n, int(ref["argmax_rank"])))


def johnson_makespan(a, b):
    """Johnson's rule for the two-machine flow shop (a first, then b)."""
    first = sorted([i for i in range(len(a)) if a[i] <= b[i]], key=lambda i: a[i])
    last = sorted([i for i in range(len(a)) if a[i] > b[i]], key=lambda i: -b[i])
    t1 = t2 = 0
    for i in first + last:
        t1 += a[i]
        t2 = max(t1, t2) + b[i]
    return t2


def test_evaluate_random_orderings_one_dma(dev):
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(500)
    for n in range(1, 17):
        for hi in (4, 1000, 20_000_000, 1 << 39):
            tasks = rng.integers(0, hi, size=(n, 3)).astype(np.int64)
            orders = np.stack([rng.permutation(n) for _ in range(400)]).astype(np.uint8)
            for m in ONE_MODELS:
                want = cmodel.eval_orders(tasks, orders, m)
                got = tgo.evaluate(to_dev(tasks, dev), to_dev(orders, dev), tmodel(m)).cpu().numpy()
                assert np.array_equal(got, want), (n, hi, m)


def test_evaluate_hand_worked_one_dma(dev):
    from paper_1806_10113_amd import tgo
    g = json.load(open(os.path.join(GOLDEN, "one_dma_hand.json")))
    for case in g["cases"]:
        tasks = np.array(case["tasks_ns"], dtype=np.int64)
        orders = np.array([case["order"]], dtype=np.uint8)
        got = tgo.evaluate(to_dev(tasks, dev), to_dev(orders, dev), tmodel(ONE)).cpu().numpy()
        assert int(got[0]) == case["T"]


def test_exhaustive_small_groups_per_ordering_one_dma(dev):
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(501)
    for n in range(1, 11):
        for hi in (3, 50_000, 20_000_000):
            tasks = rng.integers(0, hi, size=(n, 3)).astype(np.int64)
            for m in ONE_MODELS[:2]:
                ref = cmodel.exhaustive(tasks, m, per_order=True)
                summ, po = tgo.exhaustive(to_dev(tasks, dev), tmodel(m), per_order=True)
                assert np.array_equal(po.cpu().numpy(), ref["times"]), (n, hi, m)
                check_summary(tgo.read_summary(summ), ref, n)


def test_exhaustive_64bit_path_one_dma(dev):
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(502)
    for n in (4, 8):
        tasks = rng.integers(1 << 33, 1 << 39, size=(n, 3)).astype(np.int64)
        ref = cmodel.exhaustive(tasks, ONE, per_order=True)
        summ, po = tgo.exhaustive(to_dev(tasks, dev), tmodel(ONE), per_order=True)
        assert np.array_equal(po.cpu().numpy(), ref["times"])
        check_summary(tgo.read_summary(summ), ref, n)


def test_exhaustive_golden_n8_n12_one_dma(dev):
    """Stored full enumerations of the N=8 (seed 0) and N=12 mixed (seed 1)
    groups, plus 2,000 sampled N=12 orderings evaluated one by one."""
    from paper_1806_10113_amd import tgo
    gold = json.load(open(os.path.join(GOLDEN, "single_group_summaries.json")))
    for key, tasks in (("uniform_n8_seed0_one_dma", W.single_group_uniform(8, 0)),
                       ("mixed_n12_seed1_one_dma", W.single_group_mixed(12, 1))):
        g = gold[key]
        assert tasks.tolist() == g["tasks_ns"] and g["model"]["dma_engines"] == 1
        s = tgo.read_summary(tgo.exhaustive(to_dev(tasks, dev), tmodel(ONE))[0])
        check_summary(s, g, len(tasks))
    tasks = W.single_group_mixed(12, 1)
    rng = np.random.default_rng(503)
    ranks = rng.integers(0, math.factorial(12), size=2000)
    orders = np.array([M.nth_permutation(12, int(r)) for r in ranks], dtype=np.uint8)
    got = tgo.evaluate(to_dev(tasks, dev), to_dev(orders, dev), tmodel(ONE)).cpu().numpy()
    assert np.array_equal(got, cmodel.eval_orders(tasks, orders, ONE))


def test_exhaustive_n13_properties_one_dma(dev):
    """N=13 (6,227,020,800 orderings, beyond what the oracle enumerates in
    seconds): closed forms that hold at any size."""
    from paper_1806_10113_amd import tgo
    n = 13
    R = math.factorial(n)
    rng = np.random.default_rng(504)
    # no kernel work: every ordering takes sum h + sum d
    tasks = rng.integers(0, 2_000_000, size=(n, 3)).astype(np.int64)
    tasks[:, 1] = 0
    c = int(tasks[:, 0].sum() + tasks[:, 2].sum())
    s = tgo.read_summary(tgo.exhaustive(to_dev(tasks, dev), tmodel(ONE))[0])
    assert s["status"] == 0 and s["count"] == R
    assert s["min_ns"] == c and s["max_ns"] == c
    assert s["argmin_rank"] == 0 and s["argmax_rank"] == 0
    assert s["sum"] == c * R
    assert s["fingerprint"] == (c * R * R) & MASK64  # sum over r of (2r + 1) = R^2
    # no HtD work: the optimum is Johnson's two-machine flow shop on (k, d)
    tasks = rng.integers(0, 2_000_000, size=(n, 3)).astype(np.int64)
    tasks[:, 0] = 0
    s = tgo.read_summary(tgo.exhaustive(to_dev(tasks, dev), tmodel(ONE))[0])
    assert s["min_ns"] == johnson_makespan(tasks[:, 1].tolist(), tasks[:, 2].tolist())
    assert M.simulate(tasks, s["best"], ONE) == s["min_ns"]
    assert M.simulate(tasks, s["worst"], ONE) == s["max_ns"]
    # a general group: reported orderings reproduce the extremes, samples fit
    tasks = W.single_group_mixed(n, 5)
    s = tgo.read_summary(tgo.exhaustive(to_dev(tasks, dev), tmodel(ONE))[0])
    assert s["status"] == 0 and s["count"] == R
    assert M.simulate(tasks, s["best"], ONE) == s["min_ns"]
    assert M.simulate(tasks, s["worst"], ONE) == s["max_ns"]
    assert s["argmin_rank"] == M.lehmer_rank(s["best"])
    assert s["min_ns"] <= s["mean_ns"] <= s["max_ns"]
    ranks = rng.integers(0, R, size=3000)
    orders = np.array([M.nth_permutation(n, int(r)) for r in ranks], dtype=np.uint8)
    T = cmodel.eval_orders(tasks, orders, ONE)
    assert (T >= s["min_ns"]).all() and (T <= s["max_ns"]).all()
    assert s["min_ns"] <= M.simulate(tasks, M.heuristic(tasks, ONE), ONE)


def test_heuristic_batch_one_dma(dev):
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(300, 1, 16, seed=505)
    orders, ns = tgo.heuristic(to_dev(b.tasks, dev), to_dev(b.offs, dev), tmodel(ONE))
    orders, ns = orders.cpu().numpy(), ns.cpu().numpy()
    for gi in range(b.n_groups):
        tasks = b.group(gi)
        n = len(tasks)
        want = M.heuristic(tasks, ONE)
        assert list(orders[gi, :n]) == want, gi
        assert ns[gi] == M.simulate(tasks, want, ONE)


def test_batch_plan_one_dma(dev):
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(600, 1, 10, seed=506, per_task_label=True)
    tasks, offs = to_dev(b.tasks, dev), to_dev(b.offs, dev)
    plan = tgo.Plan(tmodel(ONE), max_groups=b.n_groups)
    plan.autotune(tasks, offs)
    ss = tgo.read_summaries(plan.run(tasks, offs))
    sizes = b.sizes()
    rng = np.random.default_rng(507)
    big = [g for g in range(b.n_groups) if sizes[g] >= 9]
    sample = set(rng.choice(big, size=min(12, len(big)), replace=False).tolist())
    for g in range(b.n_groups):
        grp = b.group(g)
        n = len(grp)
        assert ss[g]["status"] == 0 and ss[g]["count"] == math.factorial(n)
        if n <= 8 or g in sample:
            check_summary(ss[g], cmodel.exhaustive(grp, ONE), n)
        h = M.heuristic(grp, ONE)
        assert ss[g]["heur"] == h and ss[g]["heur_ns"] == M.simulate(grp, h, ONE)
    plan.close()


def test_random_search_one_dma(dev):
    from paper_1806_10113_amd import tgo
    ev = W.fixed_size_groups(6, 14, seed=508)
    res = tgo.read_search(tgo.random_search(to_dev(ev.tasks, dev), to_dev(ev.offs, dev), samples=256,
                                            seed=29, model=tmodel(ONE)))
    for g in range(ev.n_groups):
        grp = ev.group(g)
        orders = philox.sample_orderings(14, g, 0, 256, 29)
        T = cmodel.eval_orders(grp, orders, ONE)
        s = int(np.argmin(T))
        assert res[g]["cand_best_ns"] == T[s] and res[g]["best_sample"] == s
        h = M.simulate(grp, M.heuristic(grp, ONE), ONE)
        assert res[g]["best_ns"] == min(T[s], h)


def test_server_one_dma(dev):
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(120, 1, 10, seed=509, per_task_label=True)
    srv = tgo.Server(tmodel(ONE), tgo.server_config(streams=2, max_batch=32))
    ids = [srv.submit(b.group(g)) for g in range(b.n_groups)]
    srv.drain()
    res = {int(r["id"]): r for r in srv.poll(1000)}
    for g, i in enumerate(ids):
        grp = b.group(g)
        n = len(grp)
        r = res[i]
        assert r["status"] == 0 and r["path"] == 0
        ref = cmodel.exhaustive(grp, ONE)
        assert r["best_ns"] == ref["min_ns"]
        assert [int(v) for v in r["best"][:n]] == list(M.nth_permutation(n, ref["argmin_rank"]))
    srv.close()
