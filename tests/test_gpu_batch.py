"""GPU parity of the batched persistent path (tgo_batch) against the CPU oracle."""
import math
import os

import numpy as np
import pytest

from oracle import cmodel
from oracle import model as M
from paper_1806_10113_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def check_group(s, tasks, m, full=True):
    n = len(tasks)
    assert s["status"] == 0 and s["n"] == n
    ref = cmodel.exhaustive(tasks, m)
    for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "fingerprint"):
        assert int(s[k]) == int(ref[k]), k
    assert s["sum"] == ref["sum"]
    assert s["count"] == math.factorial(n)
    assert abs(s["mean_ns"] - ref["mean_ns"]) <= 2e-16 * ref["mean_ns"]
    assert s["best"] == list(M.nth_permutation(n, ref["argmin_rank"]))
    assert s["worst"] == list(M.nth_permutation(n, ref["argmax_rank"]))


def check_heur(s, tasks, m):
    h = M.heuristic(tasks, m)
    assert s["heur"] == h
    assert s["heur_ns"] == M.simulate(tasks, h, m)


def test_batch_small_groups_all_checked(dev):
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(240, 1, 8, seed=200, per_task_label=True)
    for m, tm in ((M.DEFAULT, tgo.DEFAULT), (M.PAPER_EXAMPLE, tgo.PAPER_EXAMPLE)):
        plan = tgo.Plan(tm, max_groups=b.n_groups)
        out = plan.run(to_dev(b.tasks, dev), to_dev(b.offs, dev))
        ss = tgo.read_summaries(out)
        for g in range(b.n_groups):
            check_group(ss[g], b.group(g), m)
            check_heur(ss[g], b.group(g), m)
        plan.close()


def test_batch_uneven_4096_groups(dev):
    """4,096 groups, N uniform in [4, 10], one DK/DT label per group, seed 2:
    every group in one persistent launch (autotuned), checked against the
    oracle on every group with N <= 8 and on a sample of the N = 9, 10 groups;
    the heuristic on every group."""
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(4096, 4, 10, seed=2)
    tasks, offs = to_dev(b.tasks, dev), to_dev(b.offs, dev)
    plan = tgo.Plan(tgo.DEFAULT, max_groups=4096)
    desc = plan.autotune(tasks, offs)
    assert desc["tuned"]
    out = plan.run(tasks, offs)
    ss = tgo.read_summaries(out)
    sizes = b.sizes()
    rng = np.random.default_rng(201)
    big = [g for g in range(b.n_groups) if sizes[g] >= 9]
    sample = set(rng.choice(big, size=16, replace=False).tolist())
    for g in range(b.n_groups):
        assert ss[g]["status"] == 0
        assert ss[g]["count"] == math.factorial(int(sizes[g]))
        if sizes[g] <= 8 or g in sample:
            check_group(ss[g], b.group(g), M.DEFAULT)
        check_heur(ss[g], b.group(g), M.DEFAULT)
        assert ss[g]["min_ns"] <= ss[g]["heur_ns"] <= ss[g]["max_ns"]
    # a fresh plan with the default decomposition gives identical bytes
    plan2 = tgo.Plan(tgo.DEFAULT, max_groups=4096)
    out2 = plan2.run(tasks, offs)
    assert bool((out2 == out).all())
    # the tuned decomposition restored into a new plan (as a later process
    # would from a saved description) is the same decomposition, same bytes
    plan3 = tgo.Plan(tgo.DEFAULT, max_groups=4096)
    plan3.set_decomposition(desc)
    d3 = plan3.describe()
    for k in ("m_by_n", "lane_mult", "blocks"):
        assert d3[k] == desc[k], k
    assert bool((plan3.run(tasks, offs) == out).all())
    bad = dict(desc, m_by_n=[1] * 11 + [6])
    with pytest.raises(tgo.TgoError):
        plan3.set_decomposition(bad)
    with pytest.raises(tgo.TgoError):
        plan3.set_decomposition(dict(desc, blocks=0))
    assert plan3.describe()["m_by_n"] == desc["m_by_n"]
    plan.close()
    plan2.close()
    plan3.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_4096_seed2.npz")


@pytest.mark.parametrize("scheme", ["two_dma", "one_dma"])
def test_batch_4096_every_group_against_stored_oracle(dev, scheme):
    """The 4,096-group batch (N uniform in [4, 10], one DK/DT label per group,
    seed 2) in one persistent launch: every field of every group equals the
    oracle's stored enumeration and Algorithm 1 (tests/golden/make_golden.py)."""
    from paper_1806_10113_amd import tgo
    gold = np.load(GOLDEN)
    b = W.batch_groups(4096, 4, 10, seed=2)
    assert (gold["sizes"] == b.sizes()).all()
    m = tgo.DEFAULT if scheme == "two_dma" else tgo.Model(2, 3, 3, 1)
    plan = tgo.Plan(m, max_groups=4096)
    out = plan.run(to_dev(b.tasks, dev), to_dev(b.offs, dev))
    ss = np.frombuffer(out.cpu().numpy().tobytes(), dtype=tgo.SUMMARY_DTYPE)
    plan.close()
    assert (ss["status"] == 0).all()
    assert (ss["n"] == b.sizes()).all()
    fact = np.array([math.factorial(int(n)) for n in b.sizes()], dtype=np.uint64)
    assert (ss["count"] == fact).all()
    for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "sum_lo", "sum_hi", "fingerprint",
              "heur_ns"):
        got = ss[k].astype(np.uint64)
        bad = np.nonzero(got != gold[f"{scheme}_{k}"])[0]
        assert len(bad) == 0, f"{k}: {len(bad)} groups differ, first {bad[:5]}"
    assert (ss["heur"] == gold[f"{scheme}_heur"]).all()
    for g in range(b.n_groups):
        n = int(b.sizes()[g])
        assert list(ss["best"][g][:n]) == list(M.nth_permutation(n, int(ss["argmin_rank"][g])))
        assert list(ss["worst"][g][:n]) == list(M.nth_permutation(n, int(ss["argmax_rank"][g])))


def test_batch_graph_replays(dev):
    """Replays of the captured graph, with eager work in between, all equal."""
    import torch
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(500, 3, 9, seed=202)
    tasks, offs = to_dev(b.tasks, dev), to_dev(b.offs, dev)
    plan = tgo.Plan(tgo.DEFAULT, max_groups=600)
    out = torch.empty((b.n_groups, tgo.SUMMARY_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    first = plan.run(tasks, offs, out).clone()
    for i in range(4):
        junk = torch.full((1 << 20,), i, dtype=torch.int64, device=dev).sum()  # eager work
        tgo.exhaustive(to_dev(W.single_group_uniform(7, i), dev))
        torch.cuda.synchronize()
        out.fill_(0xAB)
        plan.run(tasks, offs, out)
        torch.cuda.synchronize()
        assert bool((out == first).all()), f"replay {i} differs"
        del junk
    ss = tgo.read_summaries(first)
    for g in range(0, b.n_groups, 37):
        check_group(ss[g], b.group(g), M.DEFAULT)
    plan.close()


def test_batch_group_errors(dev):
    from paper_1806_10113_amd import tgo
    groups = [np.array([[1, 2, 3]] * 13, dtype=np.int64),          # n = 13: too large for a batch
              np.array([[1, -2, 3], [4, 5, 6]], dtype=np.int64),   # negative duration
              np.array([[1 << 38, 5, 6], [4, 5, 6]], dtype=np.int64),  # needs the 64-bit path
              np.array([[3, 4, 5], [6, 7, 8], [1, 1, 1]], dtype=np.int64)]
    tasks = np.concatenate(groups)
    offs = np.cumsum([0] + [len(g) for g in groups]).astype(np.int32)
    plan = tgo.Plan(tgo.DEFAULT, max_groups=8)
    ss = tgo.read_summaries(plan.run(to_dev(tasks, dev), to_dev(offs, dev)))
    assert ss[0]["status"] == tgo.TGO_EINVAL
    assert ss[1]["status"] == tgo.TGO_ERANGE
    check_group(ss[2], groups[2], M.DEFAULT)  # 64-bit path
    check_group(ss[3], groups[3], M.DEFAULT)
    with pytest.raises(tgo.TgoError):
        plan.run(to_dev(np.concatenate([tasks] * 3), dev),
                 to_dev(np.arange(0, 10 * 3, 3, dtype=np.int32), dev))  # 9 groups > max_groups
    plan.close()


@pytest.mark.parametrize("dma", [2, 1])
def test_batch_64bit_time_path(dev, dma):
    """Groups whose times pass 2^31 ns (durations up to 2^38 ns, totals near
    2^41) take the 64-bit path inside the same batch as ordinary groups;
    every group of both kinds equals the oracle, and the heuristic too."""
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(210 + dma)
    m = M.Model(4, 3, 3, dma)
    groups = []
    for i in range(40):
        n = int(rng.integers(1, 10))
        if i % 3 == 0:
            t = rng.integers(1 << 30, 1 << 38, size=(n, 3))       # 64-bit path
        elif i % 3 == 1:
            t = rng.integers(0, 3_000_000, size=(n, 3))          # 32-bit path
        else:
            t = rng.integers(0, 3_000_000, size=(n, 3))
            t[0, 1] = (1 << 31) - 1                              # one long kernel: 64-bit
        groups.append(t.astype(np.int64))
    groups.append(rng.integers(1 << 36, 1 << 38, size=(10, 3)).astype(np.int64))  # 3.6M orderings
    tasks = np.concatenate(groups)
    offs = np.cumsum([0] + [len(g) for g in groups]).astype(np.int32)
    plan = tgo.Plan(tgo.Model(2, 3, 3, dma), max_groups=64)
    ss = tgo.read_summaries(plan.run(to_dev(tasks, dev), to_dev(offs, dev)))
    for g, grp in enumerate(groups):
        check_group(ss[g], grp, m)
        check_heur(ss[g], grp, m)
    assert max(s["max_ns"] for s in ss) > (1 << 40)
    plan.close()


def test_plan_max_n_and_memory_budget(dev):
    """Groups above the plan's max_n are rejected per group; the memory
    budget bounds the plan (too small: TGO_ENOMEM) and only sets how many
    tiles a 64-bit group is cut into, not the results."""
    from paper_1806_10113_amd import tgo
    rng = np.random.default_rng(230)
    groups = [rng.integers(1, 1 << 37, size=(7, 3)).astype(np.int64),
              rng.integers(1, 3_000_000, size=(9, 3)).astype(np.int64),
              rng.integers(1, 3_000_000, size=(5, 3)).astype(np.int64)]
    tasks = np.concatenate(groups)
    offs = np.cumsum([0] + [len(g) for g in groups]).astype(np.int32)
    t, o = to_dev(tasks, dev), to_dev(offs, dev)
    small = tgo.Plan(tgo.DEFAULT, max_groups=4, max_n=8)
    ss = tgo.read_summaries(small.run(t, o))
    assert ss[1]["status"] == tgo.TGO_EINVAL
    check_group(ss[0], groups[0], M.DEFAULT)
    check_group(ss[2], groups[2], M.DEFAULT)
    tight = tgo.Plan(tgo.DEFAULT, max_groups=4, mem_budget=4096)
    assert tight.describe()["wide_tiles"] < 256
    big = tgo.Plan(tgo.DEFAULT, max_groups=4)
    a, b = tight.run(t, o), big.run(t, o)
    assert bool((a == b).all())
    with pytest.raises(tgo.TgoError) as ei:
        tgo.Plan(tgo.DEFAULT, max_groups=1000, mem_budget=1000)
    assert ei.value.code == tgo.TGO_ENOMEM
    for p in (small, tight, big):
        p.close()
