"""GPU checks of the continuous-batching server: every answer exact against
the oracle, the same alone and in a mix, admission within the memory budget
(queue rings that wrap), and a real-time replay of a Poisson trace."""
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


def check_small(r, grp):
    n = len(grp)
    assert r["status"] == 0 and r["path"] == 0 and r["n"] == n
    s = cmodel.exhaustive(grp, M.DEFAULT)
    assert r["best_ns"] == s["min_ns"]
    best = [int(v) for v in r["best"][:n]]
    assert best == list(M.nth_permutation(n, s["argmin_rank"]))
    assert r["heur_ns"] == M.simulate(grp, M.heuristic(grp, M.DEFAULT), M.DEFAULT)
    assert r["t_arrive_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]


def by_id(results):
    return {int(r["id"]): r for r in results}


def test_small_groups_exact(dev):
    from paper_1806_10113_amd import tgo
    b = W.batch_groups(300, 1, 9, seed=400, per_task_label=True)
    srv = tgo.Server(tgo.DEFAULT, tgo.server_config(streams=3, max_batch=64))
    ids = [srv.submit(b.group(g)) for g in range(b.n_groups)]
    srv.drain()
    res = by_id(srv.poll(1000))
    assert len(res) == b.n_groups
    for g, i in enumerate(ids):
        check_small(res[i], b.group(g))
    st = srv.stats()
    assert st["completed"] == b.n_groups and st["batches"] >= b.n_groups // 64
    srv.close()


def test_same_alone_and_in_mix_small_and_large(dev):
    """A request's answer does not depend on what else is in flight: the same
    small and large probes (same sampling key) alone and inside a mix."""
    from paper_1806_10113_amd import tgo
    sur = tgo.Surrogate(max_rows=1 << 14, max_groups=64)
    sur.init(9)
    cfg = tgo.server_config(streams=2, max_batch=32, max_batch_large=8, samples=4096, topk=32)
    probe_small = W.batch_groups(1, 8, 8, seed=401).group(0)
    probe_large = W.fixed_size_groups(1, 14, seed=402).group(0)
    mix = W.batch_groups(120, 4, 16, seed=403, per_task_label=True)

    def run(with_mix):
        srv = tgo.Server(tgo.DEFAULT, cfg, sur)
        ids = []
        if with_mix:
            ids += [srv.submit(mix.group(g)) for g in range(60)]
        a = srv.submit(probe_small, key=777)
        c = srv.submit(probe_large, key=778)
        if with_mix:
            ids += [srv.submit(mix.group(g)) for g in range(60, 120)]
        srv.drain()
        res = by_id(srv.poll(1000))
        srv.close()
        return res, a, c, ids

    alone, a1, c1, _ = run(False)
    mixed, a2, c2, ids = run(True)
    for x1, x2 in ((a1, a2), (c1, c2)):
        for k in ("best_ns", "heur_ns", "status", "path", "n"):
            assert alone[x1][k] == mixed[x2][k], k
        assert bytes(alone[x1]["best"]) == bytes(mixed[x2]["best"])
    check_small(alone[a1], probe_small)
    L = mixed[c2]
    assert L["path"] == 1 and L["status"] == 0
    assert L["best_ns"] == cmodel.simulate(probe_large, [int(v) for v in L["best"][:14]], M.DEFAULT)
    assert L["best_ns"] <= L["heur_ns"]
    # every mixed request is answered exactly
    for g, i in enumerate(ids):
        r = mixed[i]
        grp = mix.group(g)
        n = len(grp)
        assert r["status"] == 0
        assert r["best_ns"] == cmodel.simulate(grp, [int(v) for v in r["best"][:n]], M.DEFAULT)
        if n <= 10:
            check_small(r, grp)
        else:
            assert r["path"] == 1 and r["best_ns"] <= r["heur_ns"]
    sur.close()


TASK_BYTES = 24  # one task row: three int64 durations


def test_budget_admission(dev):
    """The budget covers the server's own device memory plus the queue rings:
    with room for about three requests' rows beyond its own memory, later
    requests wait for rows to free up, the device memory held never exceeds
    the budget, and every answer is exact (the small ring wraps many times)."""
    from paper_1806_10113_amd import tgo
    probe = tgo.Server(tgo.DEFAULT, tgo.server_config(streams=4, max_batch=16))
    base = probe.stats()["base_bytes"]
    probe.close()
    assert base > 0
    budget = base + 3 * 8 * TASK_BYTES
    cfg = tgo.server_config(streams=4, max_batch=16, budget_bytes=budget)
    b = W.batch_groups(60, 4, 8, seed=405)
    srv = tgo.Server(tgo.DEFAULT, cfg)
    st0 = srv.stats()
    assert st0["base_bytes"] == base and st0["ring_rows"][0] == 24
    assert st0["budget_bytes"] == budget
    ids = [srv.submit(b.group(g)) for g in range(b.n_groups)]
    srv.drain()
    res = by_id(srv.poll(100))
    st = srv.stats()
    assert base < st["max_in_use_bytes"] <= budget
    assert st["in_use_bytes"] == base  # everything released
    assert st["batches"] >= b.n_groups // 6
    assert st["max_queued"] > 3
    for g, i in enumerate(ids):
        check_small(res[i], b.group(g))
    srv.close()


def test_budget_below_own_memory_is_refused(dev):
    from paper_1806_10113_amd import tgo
    probe = tgo.Server(tgo.DEFAULT, tgo.server_config(streams=2, max_batch=16))
    base = probe.stats()["base_bytes"]
    probe.close()
    for budget in (1000, base, base + 9 * TASK_BYTES):  # small_max_n = 10 rows do not fit
        with pytest.raises(tgo.TgoError) as ei:
            tgo.Server(tgo.DEFAULT, tgo.server_config(streams=2, max_batch=16, budget_bytes=budget))
        assert ei.value.code == tgo.TGO_ENOMEM
    srv = tgo.Server(tgo.DEFAULT, tgo.server_config(streams=2, max_batch=16,
                                                    budget_bytes=base + 10 * TASK_BYTES))
    grp = W.batch_groups(1, 10, 10, seed=409).group(0)
    ids = [srv.submit(grp) for _ in range(3)]  # one at a time through a 10-row ring
    srv.drain()
    res = by_id(srv.poll(10))
    for i in ids:
        check_small(res[i], grp)
    srv.close()


def test_requests_larger_than_half_the_ring(dev):
    """A ring of 12 rows and groups of 7..10 tasks: a request that does not fit
    before the ring's end starts again at its beginning, and when nothing is
    held the rows it skipped count as free (no request waits forever)."""
    from paper_1806_10113_amd import tgo
    probe = tgo.Server(tgo.DEFAULT, tgo.server_config(streams=2, max_batch=8))
    base = probe.stats()["base_bytes"]
    probe.close()
    srv = tgo.Server(tgo.DEFAULT, tgo.server_config(streams=2, max_batch=8, budget_bytes=base + 12 * TASK_BYTES))
    assert srv.stats()["ring_rows"][0] == 12
    b = W.batch_groups(30, 7, 10, seed=412)
    ids = [srv.submit(b.group(g)) for g in range(b.n_groups)]
    srv.drain(30_000)
    res = by_id(srv.poll(100))
    for g, i in enumerate(ids):
        check_small(res[i], b.group(g))
    assert srv.stats()["max_in_use_bytes"] <= base + 12 * TASK_BYTES
    srv.close()


def test_large_class_ring_wraps(dev):
    """Both classes through small rings: large requests (learned proposal)
    wrap their ring and still score exactly what they report."""
    from paper_1806_10113_amd import tgo
    sur = tgo.Surrogate(max_rows=1 << 13, max_groups=8)
    sur.init(11)
    cfg = tgo.server_config(streams=2, max_batch=8, max_batch_large=4, samples=2048, topk=16)
    probe = tgo.Server(tgo.DEFAULT, cfg, sur)
    base = probe.stats()["base_bytes"]
    probe.close()
    cfg.budget_bytes = base + 3 * (10 + 16) * TASK_BYTES  # rings of 30 and 48 rows
    srv = tgo.Server(tgo.DEFAULT, cfg, sur)
    assert srv.stats()["ring_rows"] == [30, 48]
    mix = W.batch_groups(40, 6, 16, seed=410, per_task_label=True)
    ids = [srv.submit(mix.group(g)) for g in range(mix.n_groups)]
    srv.drain()
    res = by_id(srv.poll(100))
    st = srv.stats()
    assert st["max_in_use_bytes"] <= cfg.budget_bytes
    for g, i in enumerate(ids):
        grp = mix.group(g)
        n = len(grp)
        r = res[i]
        assert r["status"] == 0
        assert r["best_ns"] == cmodel.simulate(grp, [int(v) for v in r["best"][:n]], M.DEFAULT)
        if n <= 10:
            check_small(r, grp)
        else:
            assert r["path"] == 1 and r["best_ns"] <= r["heur_ns"]
    srv.close()
    sur.close()


def test_batching_window_keeps_answers(dev):
    """A batching window changes how requests are grouped into batches, not
    their answers (exhaustive: exact; learned proposal: same sampling key)."""
    from paper_1806_10113_amd import tgo
    sur = tgo.Surrogate(max_rows=1 << 13, max_groups=32)
    sur.init(13)
    mix = W.batch_groups(60, 4, 16, seed=411, per_task_label=True)
    res = []
    for win in (0, 2000):
        cfg = tgo.server_config(streams=2, max_batch=16, max_batch_large=8, samples=2048, topk=16, window_us=win)
        srv = tgo.Server(tgo.DEFAULT, cfg, sur)
        ids = [srv.submit(mix.group(g), key=1000 + g) for g in range(mix.n_groups)]
        srv.drain()
        r = by_id(srv.poll(100))
        res.append([r[i] for i in ids])
        srv.close()
    for g, (a, b) in enumerate(zip(*res)):
        for k in ("status", "path", "best_ns", "heur_ns"):
            assert a[k] == b[k], (g, k)
        assert bytes(a["best"]) == bytes(b["best"])
        if a["path"] == 0:
            check_small(a, mix.group(g))
    sur.close()


def test_replay_poisson_trace(dev):
    from paper_1806_10113_amd import tgo
    arr = W.poisson_arrivals(20_000.0, 0.1, 4, 10, seed=406)
    srv = tgo.Server(tgo.DEFAULT, tgo.server_config(streams=4, max_batch=128))
    out = srv.replay(arr.batch.tasks, arr.batch.offs, arr.t_ns)
    assert (out["status"] == 0).all()
    lat = (out["t_done_ns"] - out["t_arrive_ns"]) / 1e3
    assert (lat > 0).all()
    rng = np.random.default_rng(0)
    for g in rng.choice(arr.batch.n_groups, size=40, replace=False):
        check_small(out[g], arr.batch.group(int(g)))
    srv.close()


def test_device_error_in_a_batch_is_reported(dev, monkeypatch):
    """A completion query that reports a device error (forced from the host:
    the batch itself runs and ends normally) retires the batch with status
    TGO_EDEVICE, releases its memory, stops the server, and drain, submit and
    destroy return instead of waiting."""
    from paper_1806_10113_amd import tgo
    monkeypatch.setenv("TGO_SERVER_INJECT_QUERY_ERROR", "1")
    srv = tgo.Server(tgo.DEFAULT, tgo.server_config(streams=2, max_batch=8))
    monkeypatch.delenv("TGO_SERVER_INJECT_QUERY_ERROR")
    b = W.batch_groups(24, 4, 8, seed=407)
    ids = []
    for g in range(b.n_groups):
        try:
            ids.append(srv.submit(b.group(g)))
        except tgo.TgoError as e:  # the server may already have stopped
            assert e.code == tgo.TGO_EDEVICE
            break
    with pytest.raises(tgo.TgoError) as ei:
        srv.drain(20_000)
    assert ei.value.code == tgo.TGO_EDEVICE
    res, rc = srv.poll(100, raise_on_error=False)
    assert rc == tgo.TGO_EDEVICE
    failed = [r for r in res if r["status"] == tgo.TGO_EDEVICE]
    assert 1 <= len(failed) <= 8
    for r in res:
        if r["status"] == 0:  # batches that finished before the failure are exact
            g = ids.index(int(r["id"]))
            check_small(r, b.group(g))
    assert srv.stats()["in_use_bytes"] >= 0
    with pytest.raises(tgo.TgoError) as ei:
        srv.submit(b.group(0))
    assert ei.value.code == tgo.TGO_EDEVICE
    srv.close()  # returns: the worker does not wait for the failed slot
