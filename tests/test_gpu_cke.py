"""GPU parity of the concurrent-kernel path (tgo_evaluate_cke,
tgo_exhaustive_cke) against the oracle of oracle/cke.py and its C
transcription: hand-worked timelines, random groups under both launch
schemes and several rate models, every ordering of small groups, Algorithm 1
under the same rule, the reduction to the one-kernel-queue path, and the
errors the device reports."""
import json
import math
import os

import numpy as np
import pytest

from oracle import cke
from oracle import cmodel
from oracle import model as M
from paper_1806_10113_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MODELS = [M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN, M.Model(4, 3, 3, 1), M.Model(8, 5, 7, 2)]


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_10113_amd import tgo
    tgo.lib()
    return torch.device("cuda:0")


def to_dev(a, dev, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype=dtype))).to(dev)


def tmodel(m):
    from paper_1806_10113_amd import tgo
    return tgo.Model(int(math.log2(m.q)), m.p_htd, m.p_dth, m.dma_engines)


def test_hand_worked_timelines(dev):
    from paper_1806_10113_amd import tgo
    g = json.load(open(os.path.join(GOLDEN, "cke_hand.json")))
    m = tmodel(M.Model(**g["model"]))
    for case in g["cases"]:
        t = to_dev(np.array(case["tasks"], dtype=np.int64), dev)
        u = to_dev(case["units"], dev, np.int32)
        o = to_dev(np.array([case["order"]], dtype=np.uint8), dev)
        assert int(tgo.evaluate_cke(t, u, case["capacity"], o, m).cpu()[0]) == case["T"], case["name"]


def test_random_groups_match_the_oracle(dev):
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(501)
    for m in MODELS:
        for n in (1, 2, 3, 5, 8, 12, 16):
            tasks = rng.integers(0, 3_000_000, size=(n, 3)).astype(np.int64)
            tasks[rng.random((n, 3)) < 0.05] = 0  # some empty stages
            cap = int(rng.integers(1, 17))
            units = rng.integers(1, cap + 1, size=n).astype(np.int32)
            orders = np.array([rng.permutation(n) for _ in range(300)], dtype=np.uint8)
            got = tgo.evaluate_cke(to_dev(tasks, dev), to_dev(units, dev), cap, to_dev(orders, dev), tmodel(m))
            want = [cmodel.cke_simulate(tasks, units, cap, o, m) for o in orders]
            assert np.array_equal(got.cpu().numpy(), np.array(want)), (m, n)


@pytest.mark.parametrize("n,cap", [(1, 3), (4, 2), (6, 5), (8, 6)])
def test_exhaustive_small_groups_per_ordering(dev, n, cap):
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(502 + n)
    for m in (M.DEFAULT, M.Model(4, 3, 3, 1)):
        tasks = W.single_group_mixed(12, 40 + n)[:n]
        units = rng.integers(1, cap + 1, size=n).astype(np.int32)
        s, po = tgo.exhaustive_cke(to_dev(tasks, dev), to_dev(units, dev), cap, tmodel(m), per_order=True)
        d = tgo.read_summary(s)
        times = cmodel.cke_times(tasks, units, cap, m)
        assert np.array_equal(po.cpu().numpy(), times)
        assert d["status"] == 0 and d["count"] == math.factorial(n)
        assert d["min_ns"] == times.min() and d["argmin_rank"] == int(np.argmin(times))
        assert d["max_ns"] == times.max() and d["argmax_rank"] == int(np.argmax(times))
        assert d["sum"] == int(times.sum())
        fp = sum((2 * r + 1) * int(x) for r, x in enumerate(times)) % (1 << 64)
        assert d["fingerprint"] == fp
        h = cke.heuristic(tasks, units, cap, m)
        assert d["heur"] == h and d["heur_ns"] == cke.simulate(tasks, units, cap, h, m)
        assert d["best"] == list(M.nth_permutation(n, d["argmin_rank"]))


def test_whole_capacity_units_give_the_one_queue_results(dev):
    from paper_1806_10113_amd import tgo
    for m in (M.DEFAULT, M.Model(4, 3, 3, 1)):
        tasks = W.single_group_mixed(9, 3)
        t = to_dev(tasks, dev)
        a = tgo.read_summary(tgo.exhaustive_cke(t, to_dev([7] * 9, dev, np.int32), 7, tmodel(m))[0])
        b = tgo.read_summary(tgo.exhaustive(t, tmodel(m))[0])
        for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "sum", "fingerprint", "count"):
            assert a[k] == b[k], k
        assert a["heur"] == M.heuristic(tasks, m)


def test_n12_group_sampled_and_extremes(dev):
    """The largest group: the summary's extremes are reproduced by the oracle
    at their orderings, sampled ranks agree one by one, and every sampled time
    lies between the extremes."""
    from paper_1806_10113_amd import tgo
    n, cap = 12, 8
    tasks = W.single_group_mixed(n, 1)
    units = np.array([4, 2, 6, 3, 8, 1, 2, 5, 3, 4, 7, 2], dtype=np.int32)
    t, u = to_dev(tasks, dev), to_dev(units, dev)
    s = tgo.read_summary(tgo.exhaustive_cke(t, u, cap)[0])
    assert s["status"] == 0 and s["count"] == math.factorial(n)
    assert cmodel.cke_simulate(tasks, units, cap, s["best"], M.DEFAULT) == s["min_ns"]
    assert cmodel.cke_simulate(tasks, units, cap, s["worst"], M.DEFAULT) == s["max_ns"]
    rng = np.random.default_rng(503)
    ranks = rng.integers(0, math.factorial(n), size=2000)
    orders = np.array([M.nth_permutation(n, int(r)) for r in ranks], dtype=np.uint8)
    got = tgo.evaluate_cke(t, u, cap, to_dev(orders, dev)).cpu().numpy()
    want = np.array([cmodel.cke_simulate(tasks, units, cap, o, M.DEFAULT) for o in orders])
    assert np.array_equal(got, want)
    assert (got >= s["min_ns"]).all() and (got <= s["max_ns"]).all()
    assert s["heur"] == cke.heuristic(tasks, units, cap, M.DEFAULT)


def test_device_errors(dev):
    from paper_1806_10113_amd import tgo
    tasks = W.single_group_mixed(6, 2)
    t = to_dev(tasks, dev)
    bad_u = to_dev([1, 2, 0, 1, 1, 1], dev, np.int32)
    assert tgo.read_summary(tgo.exhaustive_cke(t, bad_u, 4)[0])["status"] == tgo.TGO_EINVAL
    big_u = to_dev([1, 2, 5, 1, 1, 1], dev, np.int32)
    assert tgo.read_summary(tgo.exhaustive_cke(t, big_u, 4)[0])["status"] == tgo.TGO_EINVAL
    neg = tasks.copy()
    neg[3, 2] = -1
    ok_u = to_dev([1, 2, 3, 1, 1, 1], dev, np.int32)
    assert tgo.read_summary(tgo.exhaustive_cke(to_dev(neg, dev), ok_u, 4)[0])["status"] == tgo.TGO_ERANGE
    orders = to_dev(np.array([[0, 1, 2, 3, 4, 5], [0, 0, 2, 3, 4, 5]], dtype=np.uint8), dev)
    out = tgo.evaluate_cke(t, ok_u, 4, orders).cpu().numpy()
    assert out[0] == cmodel.cke_simulate(tasks, [1, 2, 3, 1, 1, 1], 4, range(6), M.DEFAULT)
    assert out[1] == tgo.TGO_EINVAL
    with pytest.raises(tgo.TgoError):
        tgo.exhaustive_cke(to_dev(W.single_group_mixed(13, 1), dev), to_dev([1] * 13, dev, np.int32), 2)
    with pytest.raises(tgo.TgoError):
        tgo.exhaustive_cke(t, ok_u, 0)
