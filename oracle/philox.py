"""Counter-based random orderings (test infrastructure only).

Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): a 4 x 32-bit counter, a 2 x 32-bit key,
ten rounds of two 32x32->64 multiplications with the published multipliers,
the key bumped by the published Weyl constants between rounds.

Sampled ordering (the definition both this oracle and the GPU sampler
implement): for group g, sample s and seed, one Philox call with counter
(s mod 2^32, s >> 32, g, 0) and key (seed mod 2^32, seed >> 32) gives words
u0..u3.  A Fisher-Yates shuffle of 0..n-1 from the last position down draws,
for position i, j = hi32(x * (i + 1)) and keeps x = lo32(x * (i + 1)); x starts
at u0 and is reloaded from the next word every four draws.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def sample_ordering(n: int, g: int, s: int, seed: int):
    u = philox4x32_10((s & MASK, s >> 32, g, 0), (seed & MASK, seed >> 32))
    perm = list(range(n))
    x = u[0]
    k = 0
    for i in range(n - 1, 0, -1):
        if k and k % 4 == 0:
            x = u[k // 4]
        p = x * (i + 1)
        j = p >> 32
        x = p & MASK
        perm[i], perm[j] = perm[j], perm[i]
        k += 1
    return perm


def sample_orderings(n: int, g: int, first: int, count: int, seed: int) -> np.ndarray:
    return np.array([sample_ordering(n, g, first + i, seed) for i in range(count)], dtype=np.uint8)
