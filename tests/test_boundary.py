"""The C ABI library: loads, exports every declared symbol, rejects bad
arguments on the host (no device call is made for these)."""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

from oracle import model as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tgo.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(tgo_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1806_10113_amd import tgo
    if not os.path.exists(tgo.LIB_PATH):
        pytest.fail("libtgo.so is not built (python -m paper_1806_10113_amd.build)")
    return tgo.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert "tgo_exhaustive" in names and "tgo_evaluate" in names and "tgo_heuristic" in names
    for name in names:
        assert hasattr(L, name), name


def test_strerror_and_version(L):
    assert L.tgo_version() >= 1
    for code in (0, -1, -2, -3, -4):
        assert L.tgo_strerror(code)


def test_host_argument_errors(L):
    from paper_1806_10113_amd import tgo
    bad_models = [tgo._Model(0, 2, 3, 3), tgo._Model(3, 2, 3, 3), tgo._Model(2, 11, 3, 3),
                  tgo._Model(2, 2, 0, 3), tgo._Model(2, 2, 3, 5), tgo._Model(1, 2, 0, 3),
                  tgo._Model(1, -1, 1, 1)]
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    for m in bad_models:
        assert L.tgo_exhaustive(ctypes.byref(m), fake, 4, None, fake, None) == tgo.TGO_EINVAL
        assert L.tgo_evaluate(ctypes.byref(m), fake, 4, fake, 1, fake, None) == tgo.TGO_EINVAL
        assert L.tgo_heuristic(ctypes.byref(m), fake, fake, 1, fake, fake, None) == tgo.TGO_EINVAL
    good = tgo.DEFAULT._c()
    assert L.tgo_exhaustive(None, fake, 4, None, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_exhaustive(ctypes.byref(good), fake, 0, None, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_exhaustive(ctypes.byref(good), fake, 14, None, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_exhaustive(ctypes.byref(good), fake, 13, fake, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_exhaustive(ctypes.byref(good), None, 4, None, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_evaluate(ctypes.byref(good), fake, 17, fake, 1, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_evaluate(ctypes.byref(good), fake, 4, fake, -1, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_evaluate(ctypes.byref(good), None, 4, fake, 3, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_heuristic(ctypes.byref(good), fake, fake, -1, fake, fake, None) == tgo.TGO_EINVAL
    assert b"n must be" in L.tgo_last_error() or L.tgo_last_error()
    out = ctypes.c_int64()
    assert L.tgo_predict(None, fake, 3, fake, ctypes.byref(out)) == tgo.TGO_EINVAL
    assert L.tgo_predict(ctypes.byref(good), fake, 0, fake, ctypes.byref(out)) == tgo.TGO_EINVAL
    assert L.tgo_predict(ctypes.byref(good), fake, 17, fake, ctypes.byref(out)) == tgo.TGO_EINVAL
    assert L.tgo_predict(ctypes.byref(good), None, 3, fake, ctypes.byref(out)) == tgo.TGO_EINVAL
    # multi-round shapes: workers * rounds <= 16, (workers!)^rounds < 2^32,
    # per-ordering output only up to 12! orderings
    for T, R, po in ((0, 2, None), (2, 0, None), (9, 2, None), (13, 1, None), (7, 3, None),
                     (8, 2, fake)):
        assert L.tgo_rounds(ctypes.byref(good), fake, T, R, po, fake, None, None) == tgo.TGO_EINVAL
    assert L.tgo_rounds(ctypes.byref(good), None, 2, 2, None, fake, None, None) == tgo.TGO_EINVAL
    assert L.tgo_rounds(ctypes.byref(tgo._Model(3, 2, 3, 3)), fake, 2, 2, None, fake, None,
                        None) == tgo.TGO_EINVAL
    # device-memory limit: n in 1..12 (evaluate 1..16), capacity in 1..2^62,
    # m in 0..2^40, buffers present
    for n, cap in ((0, 10), (13, 10), (4, 0), (4, -5), (4, (1 << 62) + 1)):
        assert L.tgo_exhaustive_mem(ctypes.byref(good), fake, fake, n, cap, None, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_exhaustive_mem(ctypes.byref(good), fake, None, 4, 10, None, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_exhaustive_mem(ctypes.byref(good), None, fake, 4, 10, None, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_exhaustive_mem(None, fake, fake, 4, 10, None, fake, None) == tgo.TGO_EINVAL
    for n, cap, m in ((0, 10, 1), (17, 10, 1), (4, 0, 1), (4, 10, -1), (4, 10, (1 << 40) + 1)):
        assert L.tgo_evaluate_mem(ctypes.byref(good), fake, fake, n, cap, fake, m, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_evaluate_mem(ctypes.byref(good), fake, None, 4, 10, fake, 5, fake, None) == tgo.TGO_EINVAL
    # concurrent kernels: n in 1..12 (evaluate 1..16), capacity in 1..2^30, buffers present
    for n, cap in ((0, 4), (13, 4), (4, 0), (4, (1 << 30) + 1)):
        assert L.tgo_exhaustive_cke(ctypes.byref(good), fake, fake, n, cap, None, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_exhaustive_cke(ctypes.byref(good), fake, None, 4, 4, None, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_exhaustive_cke(None, fake, fake, 4, 4, None, fake, None) == tgo.TGO_EINVAL
    for n, cap, m in ((0, 4, 1), (17, 4, 1), (4, 0, 1), (4, 4, -1)):
        assert L.tgo_evaluate_cke(ctypes.byref(good), fake, fake, n, cap, fake, m, fake, None) == tgo.TGO_EINVAL
    assert L.tgo_evaluate_cke(ctypes.byref(good), fake, None, 4, 4, fake, 3, fake, None) == tgo.TGO_EINVAL


def test_server_config_errors(L):
    """tgo_server_create checks its configuration before touching a device."""
    from paper_1806_10113_amd import tgo
    good = tgo.DEFAULT._c()
    out = ctypes.c_void_p()
    for field, bad in (("streams", 0), ("streams", 9), ("max_batch", 0), ("max_batch_large", 5000),
                       ("small_max_n", 13), ("topk", 65), ("samples", 0), ("budget_bytes", 0),
                       ("window_us", -1), ("window_us", 100001)):
        c = tgo.server_config(**{field: bad})
        assert L.tgo_server_create(ctypes.byref(good), ctypes.byref(c), None, ctypes.byref(out)) == tgo.TGO_EINVAL, field
        assert not out.value
    c = tgo.server_config()
    assert c.window_us == 0 and c.streams == 4 and c.budget_bytes == 8 << 30
    assert L.tgo_server_create(None, ctypes.byref(c), None, ctypes.byref(out)) == tgo.TGO_EINVAL


def test_plan_decomposition_null_arguments(L):
    from paper_1806_10113_amd import tgo
    m = (ctypes.c_int32 * 12)(*([1] * 12))
    assert L.tgo_plan_set_decomposition(None, m, 1, 64) == tgo.TGO_EINVAL
    assert L.tgo_plan_set_decomposition(ctypes.c_void_p(16), None, 1, 64) == tgo.TGO_EINVAL


def test_rank_unrank_match_lexicographic_order():
    from paper_1806_10113_amd import tgo
    for n in range(1, 7):
        for r, p in enumerate(itertools.permutations(range(n))):
            assert tgo.rank(p) == r
            assert tuple(tgo.unrank(n, r)) == p
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = int(rng.integers(7, 17))
        p = list(rng.permutation(n))
        r = tgo.rank(p)
        assert r == M.lehmer_rank(p)
        assert tgo.unrank(n, r) == p
    with pytest.raises(tgo.TgoError):
        tgo.unrank(5, math.factorial(5))
    with pytest.raises(tgo.TgoError):
        tgo.rank([0, 0, 1])


def test_calibration_library_is_separate():
    """The integer issue probe lives in libtgo_probe.so (include/tgo_probe.h),
    outside the product library, and rejects bad arguments on the host."""
    from paper_1806_10113_amd import tgo
    L = tgo.lib()
    assert not hasattr(L, "tgo_valu_probe") and not hasattr(L, "tgo_probe_valu")
    path = os.path.join(os.path.dirname(tgo.LIB_PATH), "libtgo_probe.so")
    P = ctypes.CDLL(path)
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "tgo_probe.h")).read(), flags=re.S)
    for name in re.findall(r"\b(tgo_[a-z0-9_]+)\s*\(", text):
        assert hasattr(P, name), name
    P.tgo_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    fake = ctypes.c_void_p(16)
    for blocks, iters in ((0, 1), (1, 0), ((1 << 20) + 1, 1), (1, (1 << 20) + 1)):
        assert P.tgo_probe_valu(blocks, iters, fake, None) == -1
    assert P.tgo_probe_valu(1, 1, None, None) == -1
