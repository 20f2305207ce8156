"""Pins of the surrogate's oracle parts: Philox4x32-10 known-answer vectors,
the ordering sampler, the float64 network (finite differences, hand cases),
Adam's first step in closed form, and the target's lower bound."""
import itertools
import os
import math

import numpy as np
import pytest

from oracle import mlp
from oracle import model as M
from oracle import philox


def test_philox_known_answer_vectors():
    # Known-answer vectors published with the Random123 reference implementation.
    assert philox.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert philox.philox4x32_10((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2) == \
        (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert philox.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344),
                                (0xA4093822, 0x299F31D0)) == (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_sampler_is_a_near_uniform_permutation():
    n = 5
    counts = {}
    N = 24_000
    for s in range(N):
        p = tuple(philox.sample_ordering(n, 3, s, 99))
        assert sorted(p) == list(range(n))
        counts[p] = counts.get(p, 0) + 1
    assert len(counts) == math.factorial(n)
    exp = N / math.factorial(n)
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    # 119 degrees of freedom: mean 119, sd ~15.4; 200 is beyond 5 sd
    assert chi2 < 200
    # different groups, samples and seeds give different orderings
    assert philox.sample_ordering(16, 0, 1, 5) != philox.sample_ordering(16, 1, 1, 5)
    assert philox.sample_ordering(16, 0, 1, 5) != philox.sample_ordering(16, 0, 1, 6)


def test_network_hand_case():
    # 2 -> 2 -> 1: h = relu(W1 x + b1), s = w2 . h + b2
    W1 = np.array([[1.0, -2.0], [0.5, 0.25]])
    b1 = np.array([0.0, -1.0])
    W2 = np.array([[3.0, -1.0]])
    b2 = np.array([0.5])
    X = np.array([[2.0, 1.0], [1.0, 4.0]])
    # row 0: z1 = (0, 1.25-1=0.25) -> h = (0, 0.25) -> s = -0.25 + 0.5 = 0.25
    # row 1: z1 = (-7, 0.5+1-1=0.5) -> h = (0, 0.5) -> s = -0.5 + 0.5 = 0
    _, s = mlp.forward([(W1, b1), (W2, b2)], X)
    assert np.allclose(s, [0.25, 0.0])


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(7)
    params = mlp.init_params(rng, (6, 5, 4, 1))
    X = rng.normal(size=(9, 6))
    y = rng.normal(size=9)
    grads = mlp.backward(params, X, y)
    eps = 1e-6
    for li, (W, b) in enumerate(params):
        for idx in itertools.islice(np.ndindex(W.shape), 0, None, 3):
            old = W[idx]
            W[idx] = old + eps
            lp = mlp.loss(params, X, y)
            W[idx] = old - eps
            lm = mlp.loss(params, X, y)
            W[idx] = old
            assert abs((lp - lm) / (2 * eps) - grads[li][0][idx]) < 1e-6
        for i in range(len(b)):
            old = b[i]
            b[i] = old + eps
            lp = mlp.loss(params, X, y)
            b[i] = old - eps
            lm = mlp.loss(params, X, y)
            b[i] = old
            assert abs((lp - lm) / (2 * eps) - grads[li][1][i]) < 1e-6


def test_full_size_backward_spot_checks():
    rng = np.random.default_rng(8)
    params = mlp.init_params(rng)
    X = rng.uniform(0, 1, size=(16, mlp.NFEAT))
    y = rng.normal(size=16) * 0.1
    grads = mlp.backward(params, X, y)
    eps = 1e-6
    for li in range(4):
        W = params[li][0]
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in W.shape)
            old = W[idx]
            W[idx] = old + eps
            lp = mlp.loss(params, X, y)
            W[idx] = old - eps
            lm = mlp.loss(params, X, y)
            W[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grads[li][0][idx]) < 1e-5 * max(1.0, abs(fd))


def test_adam_first_step_closed_form():
    # after one step with zero moments, m_hat = g and v_hat = g^2
    g = np.array([0.3, -2.0, 1e-3])
    p = np.array([1.0, 1.0, 1.0])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-8)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_and_lower_bound():
    tasks = [(1000, 20_000_000, 0), (0, 1000, 999)]
    f = mlp.features(tasks, [1, 0])
    assert f.shape == (48,)
    assert f[0] == 0.0 and abs(f[1] - math.log1p(1.0) / mlp.SCALE) < 1e-15
    assert abs(f[4] - 1.0) < 1e-15          # 20 ms maps to 1
    assert (f[6:] == 0).all()
    rng = np.random.default_rng(9)
    for _ in range(40):
        n = int(rng.integers(1, 6))
        t = [tuple(int(v) for v in rng.integers(0, 50, 3)) for _ in range(n)]
        s = M.exhaustive(t, M.DEFAULT)
        assert mlp.lower_bound(t) <= max(s["min_ns"], 1)
        assert mlp.target(t, s["min_ns"]) >= -1e-12 or s["min_ns"] == 0


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1.0 + 2 ** -9])
    out = mlp.round_bf16(vals)
    # 8 significant bits: 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 -> 1 + 2^-6;
    # 1 + 2^-9 rounds down
    assert list(out) == [1.0, 1.0, 1.0 + 2 ** -6, -2.5, 1.0]


def test_stage_bounds_catch_planted_mistakes():
    """The stage bounds of the GPU gradient test have teeth: a weight
    gradient missing one 64-row tile of a 2,048-row batch, a transposed
    operand, a dropped mask, a bias left out and a one-position shift of the
    features are each far outside them (mistakes planted in the oracle's own
    stage values; the unaltered values, rounded to bf16 where the device
    rounds, pass)."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import mlp_stage as S
    rng = np.random.default_rng(7)
    params = mlp.init_params(rng)
    W1, b1 = mlp.round_bf16(params[0][0]), rng.normal(size=256) * 0.1
    W2 = mlp.round_bf16(params[1][0])
    rows = 2048
    X = mlp.round_bf16(rng.uniform(0, 1, size=(rows, 48)))
    e, sa = S.layer_stage(X, W1, b1, 48)
    H1 = mlp.round_bf16(e)
    S.check("h1", H1, e, S.act_bound(e, sa, 48))
    with pytest.raises(AssertionError):
        S.check("h1 without bias", mlp.round_bf16(np.maximum(X @ W1.T, 0)), e, S.act_bound(e, sa, 48))
    Xs = np.roll(X, 3, axis=1)
    with pytest.raises(AssertionError):
        e2, sa2 = S.layer_stage(Xs, W1, b1, 48)
        S.check("h1 shifted features", mlp.round_bf16(e2), e, S.act_bound(e, sa, 48))
    G2 = mlp.round_bf16(rng.normal(size=(rows, 256)) * 1e-3 * (rng.uniform(size=(rows, 256)) > 0.5))
    e, sa = S.back_stage(G2, W2, H1 > 0)
    S.check("G1", mlp.round_bf16(e), e, S.act_bound(e, sa, 256))
    with pytest.raises(AssertionError):
        S.check("G1 without mask", mlp.round_bf16(G2 @ W2), e, S.act_bound(e, sa, 256))
    with pytest.raises(AssertionError):
        S.check("G1 transposed weights", mlp.round_bf16((G2 @ W2.T) * (H1 > 0)), e, S.act_bound(e, sa, 256))
    G1 = mlp.round_bf16(e)
    e, sa = S.wgrad_stage(G1, X)
    S.check("dW1", e.astype(np.float32), e, S.sum_bound(sa, rows))
    dropped = G1[64:].T @ X[64:]
    with pytest.raises(AssertionError):
        S.check("dW1 without the first row tile", dropped, e, S.sum_bound(sa, rows))
