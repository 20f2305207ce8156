"""Stage-by-stage bounds for the network kernels (test infrastructure; uses
only the float64 oracle's definitions).

Each stage of the device's forward and backward pass is compared with the
oracle's definition of that stage applied to the device's own inputs to the
stage (the values the device stored for the previous stage), so the only
differences left are the device's own roundings in that stage:

* a float32 sum of K terms (plus a bias) is within gamma = (K + 1) 2^-24
  sum|terms| of the exact sum;
* rounding to bfloat16 moves a value by at most 2^-8 of itself;
* ReLU and the masks (h > 0, on the device's stored h) do not enlarge a
  difference.

So a stored bf16 activation must lie within gamma + 2^-8 (|exact| + gamma)
of the exact value, and a float32 reduction (a weight gradient summed over
the batch) within gamma of it.  A dropped row tile, a transposed operand, a
wrong bias or mask is far outside these bounds.
"""
from __future__ import annotations

import numpy as np

U = 2.0 ** -8
F32 = 2.0 ** -24


def act_bound(exact, sum_abs, K):
    """Bound on |stored bf16 - exact| for a float32 sum of K terms rounded to bf16."""
    gamma = (K + 1) * F32 * sum_abs
    return gamma + U * (np.abs(exact) + gamma)


def sum_bound(sum_abs, K):
    """Bound on |float32 sum - exact| for K terms."""
    return (K + 1) * F32 * sum_abs


def check(name, got, exact, bound):
    """Element-wise |got - exact| <= bound; returns the worst ratio."""
    got, exact, bound = (np.asarray(a, dtype=np.float64) for a in (got, exact, bound))
    err = np.abs(got - exact)
    bad = err > bound
    assert not bad.any(), (f"{name}: {int(bad.sum())} of {bad.size} elements outside the bound; worst "
                           f"|d| = {err[bad].max():.3e} at bound {bound[bad][np.argmax(err[bad])]:.3e}")
    ratio = err / np.maximum(bound, 1e-300)
    return float(ratio.max())


def layer_stage(A, W, b, K):
    """Exact relu(A W^T + b) and sum|terms| per element."""
    z = A @ W.T + b
    s = np.abs(A) @ np.abs(W).T + np.abs(b)
    return np.maximum(z, 0.0), s


def back_stage(G, W, mask):
    """Exact (G W) * mask and sum|terms| per element (W is [out][in])."""
    return (G @ W) * mask, (np.abs(G) @ np.abs(W)) * mask


def wgrad_stage(G, A):
    """Exact G^T A and sum|terms| per element."""
    return G.T @ A, np.abs(G).T @ np.abs(A)
