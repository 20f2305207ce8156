"""tgo_exhaustive_noalloc (scratch in a fixed per-device array, no
allocation) against tgo_exhaustive and the oracle, on consecutive calls that
shrink: the array keeps the previous call's contents, so every call must
re-initialise what it reads."""
import math

import numpy as np
import pytest

from oracle import cmodel
from oracle import model as OM

pytestmark = pytest.mark.gpu


def _run_both(tgo, torch, tasks_np, model, per_order):
    dev = torch.device("cuda:0")
    t = torch.as_tensor(tasks_np).to(dev)
    n = len(tasks_np)
    s_ref, po_ref = tgo.exhaustive(t, model, per_order=per_order)
    s_na = torch.full((tgo.SUMMARY_DTYPE.itemsize,), 0x5a, dtype=torch.uint8, device=dev)
    po_na = torch.full((math.factorial(n),), -7, dtype=torch.int64, device=dev) if per_order else None
    tgo.exhaustive_noalloc(t, s_na, po_na, model)
    torch.cuda.synchronize()
    return s_ref, po_ref, s_na, po_na


def _check_against_oracle(tgo, s, tasks_np, model, po=None):
    om = OM.Model(q=model.q, p_htd=model.p_htd, p_dth=model.p_dth, dma_engines=model.dma_engines)
    ref = cmodel.exhaustive(tasks_np, om, per_order=po is not None)
    d = tgo.read_summary(s)
    assert d["status"] == 0
    for k in ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "sum", "fingerprint", "count"):
        assert d[k] == ref[k], k
    if po is not None:
        assert np.array_equal(po.cpu().numpy(), ref["times"])


def test_noalloc_matches_exhaustive_on_shrinking_calls():
    import torch
    from paper_1806_10113_amd import tgo, workloads as W
    print("noalloc: N=12 mixed seed 1 (headline group), then N=9, N=8 64-bit path, N=7 one DMA", flush=True)
    cases = [
        (W.single_group_mixed(12, 1), tgo.DEFAULT, False),
        (W.single_group_uniform(9, 5), tgo.DEFAULT, True),
        # durations near 2^37 ns: the group takes the 64-bit time path (block partials in the scratch)
        (W.single_group_uniform(8, 6, lo=1 << 36, hi=1 << 37), tgo.Model(2, 3, 3), True),
        (W.single_group_uniform(7, 7), tgo.Model(2, 3, 3, dma_engines=1), True),
    ]
    for tasks_np, model, per_order in cases:
        s_ref, po_ref, s_na, po_na = _run_both(tgo, torch, tasks_np, model, per_order)
        assert bytes(s_na.cpu().numpy()) == bytes(s_ref.cpu().numpy()), f"summary differs at n={len(tasks_np)}"
        if per_order:
            assert torch.equal(po_na, po_ref)
        _check_against_oracle(tgo, s_na, tasks_np, model, po_na)


def test_noalloc_repeated_calls_identical_and_errors():
    import torch
    from paper_1806_10113_amd import tgo, workloads as W
    dev = torch.device("cuda:0")
    t = torch.as_tensor(W.single_group_uniform(10, 11)).to(dev)
    first = torch.empty(tgo.SUMMARY_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    tgo.exhaustive_noalloc(t, first)
    again = torch.empty_like(first)
    for _ in range(3):
        tgo.exhaustive_noalloc(t, again)
        torch.cuda.synchronize()
        assert torch.equal(first, again)
    # a negative duration is reported through the summary's status, not by a fault
    bad = W.single_group_uniform(6, 12)
    bad[2, 1] = -5
    s = torch.empty_like(first)
    tgo.exhaustive_noalloc(torch.as_tensor(bad).to(dev), s)
    torch.cuda.synchronize()
    assert tgo.read_summary(s)["status"] == tgo.TGO_ERANGE
    # host-visible argument errors
    with pytest.raises(tgo.TgoError):
        tgo.exhaustive_noalloc(torch.as_tensor(W.single_group_uniform(14, 1)).to(dev), s)
