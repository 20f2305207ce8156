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
    """Windows per subtree: n - 4 prefix windows and 4 + 12 + 24 + 24 walked."""
    cnt = opcount.Counter()
    opcount.walk_subtree(W.single_group_mixed(12, 1), 12345, 4, opcount.Rates(), cnt)
    assert cnt.windows == 8 + 64
    assert cnt.ops > 0 and cnt.events >= cnt.rate_changes >= 0
