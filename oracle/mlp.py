"""float64 reference of the surrogate network (test infrastructure only).

The surrogate scores an ordering of a task group from per-position features:
for every position p (16 positions; groups with fewer tasks are padded at the
tail with zero tasks, which leaves T unchanged) the features of the task there
are log1p(x / 1 us) / log1p(20 ms / 1 us) for x = HtD, K, DtH.  The network is
a plain multilayer perceptron 48 -> 256 -> 256 -> 256 -> 1 with ReLU between
layers; weights are stored output-major (W[out][in]).  It is trained with a
mean squared error against y = T / LB - 1, where LB is the largest of the
machine lower bounds of the group (an ordering-independent normaliser), and
Adam (Kingma and Ba, 2015).

Every function here is the textbook definition written out; sizes are generic
so small cases can be checked by hand.
"""
from __future__ import annotations

import math

import numpy as np

POS = 16
NFEAT = 3 * POS
SCALE = math.log1p(20_000.0)  # 20 ms in microseconds
LAYERS = (NFEAT, 256, 256, 256, 1)


def feature_value(x_ns):
    return np.log1p(np.asarray(x_ns, dtype=np.float64) / 1000.0) / SCALE


def features(tasks, order) -> np.ndarray:
    """48 features: (h, k, d) of the task at each position, zero past the group."""
    t = np.asarray(tasks, dtype=np.float64).reshape(-1, 3)
    f = np.zeros(NFEAT, dtype=np.float64)
    for p, x in enumerate(order):
        f[3 * p:3 * p + 3] = feature_value(t[x])
    return f


def lower_bound(tasks) -> int:
    """Largest of the machine lower bounds of any ordering of the group."""
    t = np.asarray(tasks, dtype=np.int64).reshape(-1, 3)
    h, k, d = t[:, 0], t[:, 1], t[:, 2]
    return int(max(h.sum() + (k + d).min(), h.min() + k.sum() + d.min(), (h + k).min() + d.sum(),
                   1))


def target(tasks, T) -> float:
    return float(T) / lower_bound(tasks) - 1.0


def init_params(rng: np.random.Generator, layers=LAYERS):
    """He-uniform weights, zero biases."""
    params = []
    for i in range(len(layers) - 1):
        fan_in, fan_out = layers[i], layers[i + 1]
        bound = math.sqrt(6.0 / fan_in)
        W = rng.uniform(-bound, bound, size=(fan_out, fan_in))
        b = np.zeros(fan_out)
        params.append((W, b))
    return params


def forward(params, X, round_hidden=None):
    """Activations list [X, h1, ..., hL-1] and the output column s (B,).
    round_hidden, if given, is applied to every hidden activation (to model a
    device that stores them in a narrower format)."""
    acts = [np.asarray(X, dtype=np.float64)]
    a = acts[0]
    for i, (W, b) in enumerate(params):
        z = a @ W.T + b
        if i < len(params) - 1:
            a = np.maximum(z, 0.0)
            if round_hidden is not None:
                a = round_hidden(a)
            acts.append(a)
        else:
            a = z
    return acts, a[:, 0]


def loss(params, X, y) -> float:
    _, s = forward(params, X)
    return float(np.mean((s - y) ** 2))


def backward(params, X, y, round_hidden=None):
    """Gradients of the mean squared error, [(dW, db), ...] per layer."""
    acts, s = forward(params, X, round_hidden)
    B = len(y)
    g = (2.0 / B) * (s - np.asarray(y, dtype=np.float64))  # d loss / d s
    g = g[:, None]
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        a_in = acts[i]
        grads[i] = (g.T @ a_in, g.sum(axis=0))
        if i > 0:
            g = (g @ W) * (acts[i] > 0)
    return grads


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of array p (returns new p, m, v); t counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def unflatten(p):
    """Flat float32 vector in the library's order -> [(W1, b1), ..., (W4, b4)]."""
    p = np.asarray(p, dtype=np.float64)
    out, off = [], 0
    for i in range(len(LAYERS) - 1):
        fi, fo = LAYERS[i], LAYERS[i + 1]
        W = p[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = p[off:off + fo]
        off += fo
        out.append((W, b))
    assert off == p.size
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params])


def round_bf16(a) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
