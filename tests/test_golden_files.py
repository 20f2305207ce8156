"""The stored oracle values (tests/golden/, written by make_golden.py from the
oracle alone) are consistent with the oracle on what the CPU can redo in
seconds: the reported extremes are reproduced by their orderings, counts and
means fit, and sampled groups of the stored batch are recomputed."""
import json
import math
import os

import numpy as np

from oracle import cmodel
from oracle import model as M
from paper_1806_10113_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_n13_summaries_are_self_consistent():
    g = json.load(open(os.path.join(GOLDEN, "single_group_summaries.json")))
    for key, seed in (("mixed_n13_seed7", 7), ("mixed_n13_seed1_one_dma", 1)):
        s = g[key]
        m = M.Model(s["model"]["q"], s["model"]["p_htd"], s["model"]["p_dth"], s["model"]["dma_engines"])
        tasks = W.single_group_mixed(13, seed)
        assert tasks.tolist() == s["tasks_ns"]
        assert s["count"] == math.factorial(13)
        assert s["best"] == list(M.nth_permutation(13, s["argmin_rank"]))
        assert s["worst"] == list(M.nth_permutation(13, s["argmax_rank"]))
        assert M.simulate(tasks, s["best"], m) == s["min_ns"]
        assert M.simulate(tasks, s["worst"], m) == s["max_ns"]
        assert M.simulate(tasks, s["heuristic"], m) == s["heuristic_ns"]
        assert s["heuristic"] == M.heuristic(tasks, m)
        assert s["min_ns"] <= s["heuristic_ns"] <= s["max_ns"]
        assert s["min_ns"] <= s["mean_ns"] <= s["max_ns"]
        assert abs(int(s["sum"]) / s["count"] - s["mean_ns"]) <= 1e-6 * s["mean_ns"]
        # sampled orderings lie between the stored extremes
        rng = np.random.default_rng(seed)
        orders = np.array([rng.permutation(13) for _ in range(200)], dtype=np.uint8)
        T = cmodel.eval_orders(tasks, orders, m)
        assert (T >= s["min_ns"]).all() and (T <= s["max_ns"]).all()


def test_batch_summaries_match_the_oracle_on_sampled_groups():
    gold = np.load(os.path.join(GOLDEN, "batch_4096_seed2.npz"))
    b = W.batch_groups(4096, 4, 10, seed=2)
    assert (gold["sizes"] == b.sizes()).all()
    rng = np.random.default_rng(11)
    small = [g for g in range(b.n_groups) if b.sizes()[g] <= 7]
    for scheme, m in (("two_dma", M.DEFAULT), ("one_dma", M.Model(4, 3, 3, 1))):
        for g in rng.choice(small, size=40, replace=False):
            tasks = b.group(int(g))
            s = cmodel.exhaustive(tasks, m, threads=2)
            assert gold[f"{scheme}_min_ns"][g] == s["min_ns"]
            assert gold[f"{scheme}_argmin_rank"][g] == s["argmin_rank"]
            assert gold[f"{scheme}_max_ns"][g] == s["max_ns"]
            assert gold[f"{scheme}_argmax_rank"][g] == s["argmax_rank"]
            assert int(gold[f"{scheme}_sum_lo"][g]) | (int(gold[f"{scheme}_sum_hi"][g]) << 64) == s["sum"]
            assert gold[f"{scheme}_fingerprint"][g] == s["fingerprint"]
            h = M.heuristic(tasks, m)
            assert list(gold[f"{scheme}_heur"][g][:len(h)]) == h
            assert gold[f"{scheme}_heur_ns"][g] == M.simulate(tasks, h, m)
