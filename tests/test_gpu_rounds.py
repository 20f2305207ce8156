"""GPU parity of the multi-round evaluator (Section 6.2: workers offloading
dependent tasks, NoReorder over every ordering and the proxy-driven Heuristic
setup) against the CPU oracle.  Integer results agree bit for bit."""
import json
import math
import os

import numpy as np
import pytest

from oracle import cmodel
from oracle import model as M
from oracle import rounds as RD
from paper_1806_10113_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MODELS = [M.DEFAULT, M.PAPER_EXAMPLE, M.NO_SLOWDOWN, M.Model(16, 9, 13), M.Model(4, 3, 3, 1),
          M.Model(1024, 1000, 3)]


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
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.int64))).to(dev)


def tmodel(m: M.Model):
    from paper_1806_10113_amd import tgo
    return tgo.Model(int(math.log2(m.q)), m.p_htd, m.p_dth, m.dma_engines)


def launch_seq(perms, R):
    return [w * R + r for r, p in enumerate(perms) for w in p]


def check_heuristic(s, groups, tasks, T, R, m):
    from paper_1806_10113_amd import tgo
    want, info = RD.simulate(tasks, T, R, m, perms=None, trace=True)
    assert s["heur_ns"] == want
    seq = [x for _, o in info["groups"] for x in o]
    assert s["heur"] == seq
    ends, pos = [], 0
    for _, o in info["groups"]:
        pos += len(o)
        ends.append(pos - 1)
    assert tgo.read_groups(groups) == ends


def test_hand_worked_cases(dev):
    from paper_1806_10113_amd import tgo
    g = json.load(open(os.path.join(GOLDEN, "rounds_hand.json")))
    m = M.Model(**g["model"])
    for case in g["cases"]:
        summ, po, _ = tgo.rounds(to_dev(case["tasks_ns"], dev), 2, 2, tmodel(m), per_order=True)
        assert int(po.cpu().numpy()[RD.rank(case["perms"], 2)]) == case["T"]
    for case in g["heuristic_cases"]:
        summ, _, groups = tgo.rounds(to_dev(case["tasks_ns"], dev), 2, 2, tmodel(m))
        s = tgo.read_summary(summ)
        assert s["heur_ns"] == case["T"]
        assert s["heur"] == [x for _, o in case["groups"] for x in o]


@pytest.mark.parametrize("T,R", [(1, 1), (1, 5), (2, 1), (2, 2), (2, 3), (3, 2), (3, 3), (4, 2),
                                 (2, 4), (5, 1), (4, 1), (2, 8)])
def test_every_ordering_small_shapes(dev, T, R):
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(600 + 10 * T + R)
    for hi in (4, 1000, 20_000_000):
        tasks = rng.integers(0, hi, size=(T * R, 3)).astype(np.int64)
        for m in MODELS:
            ref = RD.noreorder_summary([tuple(t) for t in tasks.tolist()], T, R, m)
            summ, po, groups = tgo.rounds(to_dev(tasks, dev), T, R, tmodel(m), per_order=True)
            s = tgo.read_summary(summ)
            assert np.array_equal(po.cpu().numpy(), np.asarray(ref["times"])), (T, R, hi, m)
            assert s["status"] == 0 and s["n"] == T * R and s["count"] == ref["count"]
            for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "fingerprint"):
                assert int(s[k]) == int(ref[k]), k
            assert s["sum"] == ref["sum"]
            assert abs(s["mean_ns"] - ref["mean_ns"]) <= 2e-16 * max(1.0, ref["mean_ns"])
            assert s["best"] == launch_seq(ref["best_perms"], R)
            assert s["worst"] == launch_seq(ref["worst_perms"], R)
            check_heuristic(s, groups, tasks.tolist(), T, R, m)


@pytest.mark.parametrize("T,R", [(4, 3), (5, 2), (3, 4)])
def test_every_ordering_many_tiles(dev, T, R):
    """13,824 / 14,400 / 1,296 orderings: many 256-lane blocks and a ragged
    last one, every ordering against the oracle."""
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(650 + 10 * T + R)
    tasks = rng.integers(0, 5_000_000, size=(T * R, 3)).astype(np.int64)
    for m in (M.DEFAULT, M.Model(4, 3, 3, 1)):
        ref = RD.noreorder_summary([tuple(t) for t in tasks.tolist()], T, R, m)
        summ, po, groups = tgo.rounds(to_dev(tasks, dev), T, R, tmodel(m), per_order=True)
        s = tgo.read_summary(summ)
        assert np.array_equal(po.cpu().numpy(), np.asarray(ref["times"])), (T, R, m)
        for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "fingerprint"):
            assert int(s[k]) == int(ref[k]), k
        assert s["sum"] == ref["sum"]
        check_heuristic(s, groups, tasks.tolist(), T, R, m)


@pytest.mark.parametrize("T,R", [(4, 4), (6, 2), (8, 1), (4, 2)])
def test_paper_shapes_sampled(dev, T, R):
    """The shapes of Section 6.2 (T = 4, 6, 8 workers; 1, 2, 4 dependent tasks)
    on benchmark tasks: every ordering against the C transcription of the
    oracle, sampled orderings against the Python oracle one by one, the
    extremes reproduced by their launch sequences, and the Heuristic setup
    exactly."""
    from paper_1806_10113_amd import tgo
    count = math.factorial(T) ** R
    rng = np.random.default_rng(700 + T)
    for bi, bk in enumerate(W.PAPER_BENCHMARKS):
        tasks = W.rounds_experiment(bk, T, R, seed=100 * T + 10 * R + bi)
        tl = [tuple(t) for t in tasks.tolist()]
        for m in (M.DEFAULT, M.Model(4, 3, 3, 1)):
            summ, po, groups = tgo.rounds(to_dev(tasks, dev), T, R, tmodel(m), per_order=True)
            s = tgo.read_summary(summ)
            got = po.cpu().numpy()
            assert s["status"] == 0 and s["count"] == count
            assert np.array_equal(got, cmodel.rounds_times(tasks, T, R, m)), (bk, m)
            for rk in rng.integers(0, count, size=40):
                want = RD.simulate(tl, T, R, m, perms=RD.unrank(T, R, int(rk)))
                assert int(got[rk]) == want, (bk, m, int(rk))
            assert int(got.min()) == s["min_ns"] and int(got.max()) == s["max_ns"]
            assert int(np.argmin(got)) == s["argmin_rank"] and int(np.argmax(got)) == s["argmax_rank"]
            assert s["sum"] == int(got.astype(object).sum())
            fp = sum((2 * r + 1) * int(v) for r, v in enumerate(got.tolist())) % (1 << 64)
            assert s["fingerprint"] == fp
            best = RD.unrank(T, R, s["argmin_rank"])
            assert s["best"] == launch_seq(best, R)
            assert RD.simulate(tl, T, R, m, perms=best) == s["min_ns"]
            assert RD.simulate(tl, T, R, m, perms=RD.unrank(T, R, s["argmax_rank"])) == s["max_ns"]
            check_heuristic(s, groups, tl, T, R, m)


def test_errors(dev):
    from paper_1806_10113_amd import tgo
    tasks = np.array([[1, 2, 3], [4, -5, 6], [7, 8, 9], [1, 1, 1]], dtype=np.int64)
    s = tgo.read_summary(tgo.rounds(to_dev(tasks, dev), 2, 2)[0])
    assert s["status"] == tgo.TGO_ERANGE and s["heur_ns"] == tgo.TGO_ERANGE
    big = tasks.copy()
    big[0, 0] = 1 << 40
    s = tgo.read_summary(tgo.rounds(to_dev(big, dev), 2, 2)[0])
    assert s["status"] == tgo.TGO_ERANGE
