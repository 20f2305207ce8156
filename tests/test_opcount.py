"""The operation-count transcription (opcount.py) walks the same orderings
with the same times as the oracle, so the counts it reports belong to the
method as it is computed."""
import math

import numpy as np

import opcount
from oracle import model as M
from paper_1806_10113_amd import workloads as W


def test_transcription_times_equal_the_oracle():
    rng = np.random.default_rng(3)
    r = opcount.Rates()
    for tasks, n in ((W.single_group_mixed(12, 1), 12), (W.single_group_uniform(8, 0), 8)):
        nsub = math.factorial(n) // 24
        for sub in rng.choice(nsub, size=20, replace=False):
            ts = opcount.walk_subtree(tasks, int(sub), 4, r, opcount.Counter())
            assert len(ts) == 24
            for l, T in enumerate(ts):
                rank = int(sub) * 24 + l
                assert T == M.simulate(tasks, M.nth_permutation(n, rank), M.DEFAULT), (n, rank)


def test_counts_per_subtree():
    """Windows per subtree: n - 4 prefix windows and 4 + 12 + 24 + 24 walked (M = 4)."""
    cnt = opcount.Counter()
    opcount.walk_subtree(W.single_group_mixed(12, 1), 12345, 4, opcount.Rates(), cnt)
    assert cnt.windows == 8 + 64
    assert cnt.ops > 0 and cnt.events >= cnt.rate_changes >= 0


def test_chain_form_matches_the_oracle_on_random_groups():
    """The chain form (each DtH's start and end appended once its kernel's end
    is known; windows cross only the DtHs that end inside them) gives the
    oracle's T for whole orderings, across rates (q = 1, p = q, p = 1, q up
    to 16), zero durations and groups up to 8 tasks."""
    rng = np.random.default_rng(17)
    rates = ((2, 3, 3), (0, 1, 1), (1, 1, 2), (2, 4, 4), (3, 5, 7), (4, 16, 9), (3, 1, 8))
    for trial in range(300):
        n = int(rng.integers(1, 9))
        hi = (5, 50, 10 ** 6)[trial % 3]
        tasks = rng.integers(0, hi, size=(n, 3))
        order = [int(x) for x in rng.permutation(n)]
        for q_log2, p_h, p_d in rates:
            r = opcount.Rates(q_log2, p_h, p_d)
            H, D = opcount.tables(tasks.tolist(), r)
            s = opcount.Lane(n)
            cnt = opcount.Counter()
            for j, x in enumerate(order):
                opcount.window(s, j, x, H, D, r, j < n - 1, cnt)
            T = opcount.tail(s, r, cnt)
            ref = M.simulate(tasks.tolist(), order, M.Model(1 << q_log2, p_h, p_d, 2))
            assert T == ref, (tasks.tolist(), order, (q_log2, p_h, p_d))
