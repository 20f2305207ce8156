"""GPU checks of the learned proposal: sampler and exact pairs bit for bit,
network scores and gradients against the float64 oracle within the error the
bfloat16 storage allows, training progress, search results checked exactly,
and the gain of the trained network over random candidates."""
import numpy as np
import pytest

import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import cmodel
from oracle import mlp
from oracle import model as M
from oracle import philox
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


def oracle_features(b, orders, gid):
    X = np.zeros((len(gid), mlp.NFEAT))
    for i, (o, g) in enumerate(zip(orders, gid)):
        n = b.sizes()[g]
        X[i] = mlp.features(b.group(g), [int(v) for v in o[:n]])
    return X


def test_pairs_sampler_and_exact_times(dev):
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(40, 8, 16, seed=300, per_task_label=True)
    orders, gid, T, status = tgo.pairs(to_dev(b.tasks, dev), to_dev(b.offs, dev), 128, seed=11)
    orders, gid, T = orders.cpu().numpy(), gid.cpu().numpy(), T.cpu().numpy()
    assert (status.cpu().numpy() == 0).all()
    for g in range(b.n_groups):
        n = b.sizes()[g]
        rows = slice(g * 128, (g + 1) * 128)
        assert (gid[rows] == g).all()
        want = philox.sample_orderings(n, g, 0, 128, 11)
        assert np.array_equal(orders[rows, :n], want)
        assert (orders[rows, n:] == 0xFF).all()
        assert np.array_equal(T[rows], cmodel.eval_orders(b.group(g), want, M.DEFAULT))


def setup_net(seed):
    rng = np.random.default_rng(seed)
    params = mlp.init_params(rng)
    flat = mlp.flatten(params).astype(np.float32)
    return flat


def test_scores_against_float64_oracle(dev):
    import torch
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(16, 8, 16, seed=301, per_task_label=True)
    tasks, offs = to_dev(b.tasks, dev), to_dev(b.offs, dev)
    orders, gid, T, _ = tgo.pairs(tasks, offs, 64, seed=12)
    sur = tgo.Surrogate(max_rows=4096, max_groups=64)
    flat = setup_net(1)
    sur.set_params(flat)
    got = sur.score(tasks, offs, orders, gid).cpu().numpy().astype(np.float64)
    # device: bf16 inputs, weights and hidden activations, float32 sums
    params = [(mlp.round_bf16(Wt), bb) for Wt, bb in mlp.unflatten(flat)]
    params[-1] = (mlp.unflatten(flat)[-1][0], mlp.unflatten(flat)[-1][1])  # head kept in float32
    X = mlp.round_bf16(oracle_features(b, orders.cpu().numpy(), gid.cpu().numpy()))
    _, want = mlp.forward(params, X, round_hidden=mlp.round_bf16)
    err = np.abs(got - want)
    scale = np.maximum(1.0, np.abs(want))
    # a hidden value near a bf16 rounding boundary may round the other way
    # (one ulp = 2^-8 relative); allow 2% of scale per score, 0.2% typical
    assert (err <= 2e-2 * scale).all(), err.max()
    assert np.median(err / scale) < 2e-3
    sur.close()


def _grad_case(dev, rows_groups, per, seed_groups, seed_pairs, seed_net):
    import torch
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(rows_groups, 8, 16, seed=seed_groups, per_task_label=True)
    tasks, offs = to_dev(b.tasks, dev), to_dev(b.offs, dev)
    orders, gid, T, _ = tgo.pairs(tasks, offs, per, seed=seed_pairs)
    sur = tgo.Surrogate(max_rows=8192, max_groups=4096)
    flat = setup_net(seed_net)
    sur.set_params(flat)
    grad, loss = sur.grad(tasks, offs, orders, gid, T)
    return sur, b, flat, orders.cpu().numpy(), gid.cpu().numpy(), T.cpu().numpy(), grad.cpu().numpy(), \
        float(loss.cpu()[0])


@pytest.mark.parametrize("groups,per", [(32, 64), (4, 64), (96, 64)])
def test_gradients_stage_by_stage(dev, groups, per):
    """Every stage of the device's forward and backward pass, element by
    element, against the oracle's definition of that stage on the device's
    own stage inputs (bounds in tests/mlp_stage.py): features, h1, h2, h3,
    scores, the three activation gradients, every weight and bias gradient
    and the loss.  Batches of 256 (8 row blocks), 2,048 and 6,144 rows."""
    import mlp_stage as S
    sur, b, flat, on, og, Tn, grad, loss = _grad_case(dev, groups, per, 302, 13, 2)
    rows = len(og)
    P = mlp.unflatten(flat)
    W1, b1 = mlp.round_bf16(P[0][0]), P[0][1]
    W2, b2 = mlp.round_bf16(P[1][0]), P[1][1]
    W3, b3 = mlp.round_bf16(P[2][0]), P[2][1]
    w4, b4 = P[3][0][0], P[3][1][0]
    X = sur.batch_values(sur.BATCH_FEATURES, rows)
    H1 = sur.batch_values(sur.BATCH_H1, rows)
    H2 = sur.batch_values(sur.BATCH_H2, rows)
    H3 = sur.batch_values(sur.BATCH_H3, rows)
    sc = sur.batch_values(sur.BATCH_SCORE, rows).astype(np.float64)
    G3 = sur.batch_values(sur.BATCH_G3, rows)
    G2 = sur.batch_values(sur.BATCH_G2, rows)
    G1 = sur.batch_values(sur.BATCH_G1, rows)
    # features: one float32 then one bf16 rounding of the float64 value
    Xo = oracle_features(b, on, og)
    # float32 evaluation on the device (conversion, scaling, log1pf, 1/scale:
    # a few ulp), then one bf16 rounding
    S.check("features", X, Xo, (S.U + 16 * S.F32) * np.abs(Xo))
    # forward stages on the device's own inputs
    e, sa = S.layer_stage(X, W1, b1, 48)
    S.check("h1", H1, e, S.act_bound(e, sa, 48))
    e, sa = S.layer_stage(H1, W2, b2, 256)
    S.check("h2", H2, e, S.act_bound(e, sa, 256))
    e, sa = S.layer_stage(H2, W3, b3, 256)
    S.check("h3", H3, e, S.act_bound(e, sa, 256))
    e = H3 @ w4 + b4
    S.check("score", sc, e, S.sum_bound(np.abs(H3) @ np.abs(w4) + abs(b4), 256))
    # loss gradient on the device's scores; targets y = T / LB - 1 (float32 on the device)
    y = np.array([mlp.target(b.group(g), t) for g, t in zip(og, Tn)])
    ds = 2.0 * (sc - y) / rows
    dds = 2.0 / rows * 6 * S.F32 * (np.abs(sc) + np.abs(y))
    e = (H3 > 0) * (ds[:, None] * w4[None, :])
    S.check("G3", G3, e, (S.U + 2 * S.F32) * np.abs(e) + (H3 > 0) * (dds[:, None] * np.abs(w4)[None, :]) * (1 + S.U)
            + 1e-45)
    e, sa = S.back_stage(G3, W3, H2 > 0)
    S.check("G2", G2, e, S.act_bound(e, sa, 256))
    e, sa = S.back_stage(G2, W2, H1 > 0)
    S.check("G1", G1, e, S.act_bound(e, sa, 256))
    # gradients: float32 sums over the batch of the device's stored values
    want, bnd = [], []
    for G, A in ((G1, X), (G2, H1), (G3, H2)):
        e, sa = S.wgrad_stage(G, A)
        want.append((e, G.sum(axis=0)))
        bnd.append((S.sum_bound(sa, rows), S.sum_bound(np.abs(G).sum(axis=0), rows)))
    e4 = (ds[:, None] * H3).sum(axis=0)
    bnd4 = S.sum_bound(np.abs(ds) @ np.abs(H3), rows) + dds @ np.abs(H3)
    want.append((e4[None, :], np.array([ds.sum()])))
    bnd.append((bnd4[None, :], np.array([S.sum_bound(np.abs(ds).sum(), rows) + dds.sum()])))
    S.check("gradient", grad, mlp.flatten(want), mlp.flatten(bnd))
    lo = np.mean((sc - y) ** 2)
    assert abs(loss - lo) <= S.sum_bound(np.sum((sc - y) ** 2) / rows, rows) + 8 * S.F32 * lo + 1e-12
    # and, as a whole, the device gradient follows the float64 network (no
    # bf16 anywhere but the weights and inputs): direction and size per block
    params = [(mlp.round_bf16(Wt), bb) for Wt, bb in P]
    params[-1] = P[-1]
    full = mlp.flatten(mlp.backward(params, mlp.round_bf16(Xo), y, round_hidden=mlp.round_bf16))
    off = 0
    for fi, fo in zip(mlp.LAYERS[:-1], mlp.LAYERS[1:]):
        for size in (fo * fi, fo):
            a, wv = grad[off:off + size].astype(np.float64), full[off:off + size]
            off += size
            rel = np.linalg.norm(a - wv) / max(np.linalg.norm(wv), 1e-12)
            cos = float(a @ wv) / max(np.linalg.norm(a) * np.linalg.norm(wv), 1e-30)
            assert rel < 0.05 and cos > 0.998, (fi, fo, size, rel, cos)
    sur.close()


def test_adam_step_against_oracle(dev):
    """tgo_surrogate_adam_step against the oracle's Adam (float64) from the
    device's own previous state, three steps, element by element: m and v
    within 2^-22 of their terms, the parameters within 2^-23 of themselves
    plus 2^-20 of the update (float32 evaluation of the same formula)."""
    import torch
    from paper_1806_10113_amd import tgo
    sur = tgo.Surrogate(max_rows=1024, max_groups=16)
    flat = setup_net(3)
    sur.set_params(flat)
    rng = np.random.default_rng(5)
    N = tgo.SURROGATE_PARAMS
    p_prev = sur.get_params().astype(np.float64)
    m_prev, v_prev, t0 = sur.moments()
    assert t0 == 0 and not m_prev.any() and not v_prev.any()
    m_prev, v_prev = m_prev.astype(np.float64), v_prev.astype(np.float64)
    for t, lr in ((1, 1e-3), (2, 3e-4), (3, 1e-3)):
        g = (rng.normal(size=N) * 10.0 ** rng.uniform(-6, 0, size=N)).astype(np.float32)
        g[::97] = 0.0
        sur.adam_step(torch.as_tensor(g).to(dev), lr)
        p_dev = sur.get_params().astype(np.float64)
        m_dev, v_dev, step = sur.moments()
        assert step == t
        lr32 = float(np.float32(lr))
        p_or, m_or, v_or = mlp.adam_step(p_prev, g.astype(np.float64), m_prev, v_prev, t, lr32)
        assert (np.abs(m_dev - m_or) <= 2.0 ** -22 * (0.9 * np.abs(m_prev) + 0.1 * np.abs(g)) + 1e-45).all()
        assert (np.abs(v_dev - v_or) <= 2.0 ** -22 * (0.999 * v_prev + 0.001 * g.astype(np.float64) ** 2)
                + 1e-45).all()
        upd = np.abs(p_or - p_prev)
        assert (np.abs(p_dev - p_or) <= 2.0 ** -23 * np.abs(p_or) + 2.0 ** -20 * upd + 1e-45).all()
        # the first step moves every parameter with a nonzero gradient by lr (Adam's closed form)
        if t == 1:
            nz = g != 0
            assert np.allclose(upd[nz], lr32 * np.abs(g[nz]) / (np.abs(g[nz]) + 1e-8), rtol=1e-5)
            assert (p_dev[~nz] == p_prev[~nz]).all()
        p_prev, m_prev, v_prev = p_dev, m_dev.astype(np.float64), v_dev.astype(np.float64)
    sur.close()


def test_train_step_is_grad_then_adam(dev):
    """train_step on a batch gives bit for bit the parameters of grad() on the
    same batch followed by adam_step with that gradient."""
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(24, 8, 16, seed=310, per_task_label=True)
    tasks, offs = to_dev(b.tasks, dev), to_dev(b.offs, dev)
    orders, gid, T, _ = tgo.pairs(tasks, offs, 128, seed=15)
    flat = setup_net(4)
    a = tgo.Surrogate(max_rows=4096, max_groups=64)
    c = tgo.Surrogate(max_rows=4096, max_groups=64)
    a.set_params(flat)
    c.set_params(flat)
    for step in range(3):
        la = a.train_step(tasks, offs, orders, gid, T, lr=1e-3)
        g, lc = c.grad(tasks, offs, orders, gid, T)
        c.adam_step(g, 1e-3)
        assert float(la.cpu()[0]) == float(lc.cpu()[0])
        assert np.array_equal(a.get_params(), c.get_params()), step
    a.close()
    c.close()


def trained(dev, steps=600, seed=5, groups=256):
    import torch
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(groups, 10, 16, seed=1003, per_task_label=True)
    tasks, offs = to_dev(b.tasks, dev), to_dev(b.offs, dev)
    orders, gid, T, status = tgo.pairs(tasks, offs, 512, seed=17)
    sur = tgo.Surrogate(max_rows=1 << 16, max_groups=4096)
    sur.init(seed)
    P = orders.shape[0]
    g = torch.Generator(device="cpu").manual_seed(0)
    losses = []
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    for step in range(steps):
        idx = torch.randint(0, P, (4096,), generator=g).to(dev)
        sur.train_step(tasks, offs, orders[idx].contiguous(), gid[idx].contiguous(), T[idx].contiguous(),
                       lr=1e-3 if step < steps // 2 else 3e-4, loss=loss)
        if step % 50 == 0 or step == steps - 1:
            losses.append(float(loss.cpu()[0]))
    return sur, losses


def test_training_reduces_loss(dev):
    sur, losses = trained(dev, steps=400)
    assert losses[-1] < 0.5 * losses[0], losses
    sur.close()


def test_search_results_exact_and_better_than_random_candidates(dev):
    from paper_1806_10113_amd import tgo
    sur, _ = trained(dev, steps=3000, groups=1024)
    ev = W.fixed_size_groups(48, 16, seed=3)
    tasks, offs = to_dev(ev.tasks, dev), to_dev(ev.offs, dev)
    res = tgo.read_search(sur.search(tasks, offs, samples=20_000, topk=64, seed=21))
    rnd = tgo.read_search(tgo.random_search(tasks, offs, samples=64, seed=22))
    wins = 0
    for g in range(ev.n_groups):
        r = res[g]
        grp = ev.group(g)
        assert r["status"] == 0
        assert sorted(r["best"]) == list(range(16))
        assert r["best_ns"] == cmodel.simulate(grp, r["best"], M.DEFAULT)
        assert r["heur_ns"] == M.simulate(grp, M.heuristic(grp, M.DEFAULT), M.DEFAULT)
        assert r["best_ns"] <= r["heur_ns"] and r["best_ns"] <= r["cand_best_ns"]
        if r["from_heuristic"] == 0:
            perm = philox.sample_ordering(16, g, r["best_sample"], 21)
            assert perm == r["best"]
        wins += r["cand_best_ns"] < rnd[g]["cand_best_ns"]
    # the network's 64 candidates beat 64 uniformly sampled ones on most
    # groups; if the network were no better than chance, 34 or more wins of 48
    # would happen with probability below 0.3% (one-sided binomial)
    assert wins >= 34, wins
    sur.close()


def test_random_search_matches_oracle(dev):
    from paper_1806_10113_amd import tgo
    ev = W.fixed_size_groups(6, 12, seed=303)
    res = tgo.read_search(tgo.random_search(to_dev(ev.tasks, dev), to_dev(ev.offs, dev), samples=256,
                                            seed=23))
    for g in range(ev.n_groups):
        grp = ev.group(g)
        orders = philox.sample_orderings(12, g, 0, 256, 23)
        T = cmodel.eval_orders(grp, orders, M.DEFAULT)
        s = int(np.argmin(T))
        assert res[g]["cand_best_ns"] == T[s] and res[g]["best_sample"] == s
        h = M.simulate(grp, M.heuristic(grp, M.DEFAULT), M.DEFAULT)
        assert res[g]["best_ns"] == min(T[s], h)


@pytest.mark.parametrize("n,groups,tiles", [(8, 3, 65539), (7, 16, 262147)])
def test_random_search_many_samples_exact(dev, n, groups, tiles):
    # millions of samples per group (several 64-sample tiles per wave, the
    # last chunk of each group ragged): with n! small beside the sample
    # count an optimal ordering is all but surely drawn, so the result is
    # fixed exactly: the optimum over all n! orderings (brute force) and the
    # first sample index that draws an optimal ordering
    import itertools
    from paper_1806_10113_amd import tgo
    ev = W.fixed_size_groups(groups, n, seed=305 + n)
    samples = tiles * 64 - 5                      # rounded up to tiles * 64
    res = tgo.read_search(tgo.random_search(to_dev(ev.tasks, dev), to_dev(ev.offs, dev), samples=samples,
                                            seed=24))
    allp = np.array(list(itertools.permutations(range(n))), dtype=np.uint8)
    for g in range(groups):
        grp = ev.group(g)
        T = cmodel.eval_orders(grp, allp, M.DEFAULT)
        best = int(T.min())
        optimal = {tuple(int(v) for v in p) for p in allp[T == best]}
        s = 0
        while tuple(philox.sample_ordering(n, g, s, 24)) not in optimal:
            s += 1
        assert s < tiles * 64
        assert res[g]["cand_best_ns"] == best and res[g]["best_sample"] == s, (g, res[g], best, s)


def test_save_load_roundtrip(dev, tmp_path):
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(8, 8, 16, seed=304, per_task_label=True)
    tasks, offs = to_dev(b.tasks, dev), to_dev(b.offs, dev)
    orders, gid, T, _ = tgo.pairs(tasks, offs, 64, seed=14)
    a = tgo.Surrogate(max_rows=1024, max_groups=16)
    a.init(5)
    path = str(tmp_path / "net.bin")
    a.save(path)
    raw = open(path, "rb").read()
    assert raw[:8] == b"TGOSURR1" and len(raw) == 16 + 4 * tgo.SURROGATE_PARAMS
    c = tgo.Surrogate(max_rows=1024, max_groups=16)
    c.init(6)
    c.load(path)
    assert np.array_equal(a.get_params(), c.get_params())
    sa = a.score(tasks, offs, orders, gid).cpu().numpy()
    sc = c.score(tasks, offs, orders, gid).cpu().numpy()
    assert np.array_equal(sa, sc)
    bad = tmp_path / "bad.bin"
    bad.write_bytes(raw[:-4])
    with pytest.raises(tgo.TgoError):
        c.load(str(bad))
    bad.write_bytes(b"XXXXXXXX" + raw[8:])
    with pytest.raises(tgo.TgoError):
        c.load(str(bad))
    a.close()
    c.close()


def _orderable(scores: np.ndarray) -> np.ndarray:
    """float32 -> uint32 with the same order (the search's key bits)."""
    u = np.asarray(scores, dtype=np.float32).view(np.uint32).astype(np.uint64)
    neg = (u & 0x80000000) != 0
    return np.where(neg, (~u) & 0xFFFFFFFF, u | 0x80000000)


@pytest.mark.parametrize("samples,topk", [(5000, 64), (1024, 17), (40, 64), (2049, 1)])
def test_candidates_are_the_k_lowest_scores(dev, samples, topk):
    """The search's candidate set is exactly the topk lowest network scores of
    the group's sampled orderings, ties to the lower sample index: the same
    samples (drawn by the oracle's Philox) are scored through
    tgo_surrogate_score and sorted on the host.  Covers several 1,024-key
    runs with a ragged last run, a single run, fewer samples than topk, and
    topk = 1."""
    import torch
    from paper_1806_10113_amd import tgo
    ev = W.fixed_size_groups(5, 16, seed=306)
    small = W.batch_groups(3, 9, 15, seed=307, per_task_label=True)
    sizes = list(ev.sizes()) + list(small.sizes())
    tasks_np = np.concatenate([ev.tasks, small.tasks])
    offs_np = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    tasks, offs = to_dev(tasks_np, dev), to_dev(offs_np, dev)
    G = len(sizes)
    sur = tgo.Surrogate(max_rows=1 << 15, max_groups=64)
    sur.init(8)
    cand = sur.candidates(tasks, offs, samples=samples, topk=topk, seed=41).cpu().numpy().view(np.uint64)
    for g in range(G):
        n = sizes[g]
        orders = philox.sample_orderings(n, g, 0, samples, 41)
        full = np.full((samples, 16), 0xFF, dtype=np.uint8)
        full[:, :n] = orders
        sc = sur.score(tasks, offs, to_dev(full, dev), to_dev(np.full(samples, g, dtype=np.int32), dev))
        sc = sc.cpu().numpy()
        keys = (_orderable(sc) << np.uint64(32)) | np.arange(samples, dtype=np.uint64)
        want = np.sort(keys)[:topk]
        got = cand[g]
        k = min(topk, samples)
        assert np.array_equal(got[:k], want[:k]), g
        assert (got[k:] == np.uint64(0xFFFFFFFFFFFFFFFF)).all()
    sur.close()


def _wide_batch(seed):
    """Groups on the 64-bit time path (durations up to 2^38 ns) between
    ordinary ones."""
    rng = np.random.default_rng(seed)
    groups = []
    for i in range(12):
        n = int(rng.integers(6, 17))
        hi = (1 << 38) if i % 2 == 0 else 3_000_000
        groups.append(rng.integers(1, hi, size=(n, 3)).astype(np.int64))
    tasks = np.concatenate(groups)
    offs = np.cumsum([0] + [len(g) for g in groups]).astype(np.int32)
    return groups, tasks, offs


def test_64bit_time_path_in_pairs_and_searches(dev):
    """Groups whose times pass 2^31 ns: exact pairs, the plain search (best
    sample and time against the oracle's evaluation of every sample) and the
    learned-proposal search (exact re-score of its own candidates)."""
    from paper_1806_10113_amd import tgo
    groups, tasks_np, offs_np = _wide_batch(320)
    tasks, offs = to_dev(tasks_np, dev), to_dev(offs_np, dev)
    orders, gid, T, status = tgo.pairs(tasks, offs, 64, seed=18)
    assert (status.cpu().numpy() == 0).all()
    on, Tn = orders.cpu().numpy(), T.cpu().numpy()
    for g, grp in enumerate(groups):
        n = len(grp)
        rows = slice(g * 64, (g + 1) * 64)
        assert np.array_equal(Tn[rows], cmodel.eval_orders(grp, on[rows, :n], M.DEFAULT)), g
    assert Tn.max() > (1 << 40)
    res = tgo.read_search(tgo.random_search(tasks, offs, samples=3000, seed=25))
    for g, grp in enumerate(groups):
        n = len(grp)
        smp = philox.sample_orderings(n, g, 0, 3008, 25)  # rounded up to 64-sample tiles
        Ts = cmodel.eval_orders(grp, smp, M.DEFAULT)
        s = int(np.argmin(Ts))
        assert res[g]["status"] == 0
        assert res[g]["cand_best_ns"] == Ts[s] and res[g]["best_sample"] == s, g
        h = M.simulate(grp, M.heuristic(grp, M.DEFAULT), M.DEFAULT)
        assert res[g]["heur_ns"] == h and res[g]["best_ns"] == min(int(Ts[s]), h)
    sur = tgo.Surrogate(max_rows=1 << 14, max_groups=64)
    sur.init(12)
    out = tgo.read_search(sur.search(tasks, offs, samples=2048, topk=16, seed=26))
    cand = sur.candidates(tasks, offs, samples=2048, topk=16, seed=26).cpu().numpy().view(np.uint64)
    for g, grp in enumerate(groups):
        n = len(grp)
        smp = [int(k) & 0xFFFFFFFF for k in cand[g]]
        perms = np.array([philox.sample_ordering(n, g, s, 26) for s in smp], dtype=np.uint8)
        Ts = cmodel.eval_orders(grp, perms, M.DEFAULT)
        i = min(range(len(smp)), key=lambda j: (int(Ts[j]), smp[j]))
        r = out[g]
        assert r["status"] == 0 and r["cand_best_ns"] == Ts[i] and r["best_sample"] == smp[i], g
        assert r["best_ns"] == cmodel.simulate(grp, r["best"], M.DEFAULT)
    sur.close()
