"""The 32-bit time path divides by an overlap-rate numerator p (1..1024) with
one fused multiply-add in double precision: ceil(u / p) is taken as
trunc(fma(u, 1/p, (p - 1/2)/p)) for work amounts u < 2^32, with the two
constants rounded to double on the host as 1.0 / p and (p - 0.5) * (1.0 / p).

The exact value (u + p - 1/2) / p sits at least 1/(2p) away from the
integers that bracket ceil(u/p), so the shortcut is exact whenever the
rounding error of the two constants and of the one final rounding stays
below 1/(2p).  These tests bound that error exactly (rational arithmetic)
for every p, and evaluate the shortcut itself, with the fused multiply-add
emulated exactly (the exact rational product-sum rounded once to the
nearest double), at the work amounts where it is closest to failing:
u = k p and k p + 1 (distance 1/(2p) to an integer), and k p - 1."""
import math
from fractions import Fraction

import numpy as np
import pytest

U_MAX = 1 << 32


def constants(p: int):
    inv = 1.0 / p          # rounded to nearest, as the host computes it
    c = (p - 0.5) * inv    # one more rounding, as the host computes it
    return inv, c


def shortcut(u: int, p: int) -> int:
    inv, c = constants(p)
    exact = Fraction(u) * Fraction(inv) + Fraction(c)
    return math.trunc(float(exact))  # float(Fraction) rounds to nearest even once


def test_error_bound_below_half_over_p_for_every_p():
    half_ulp_at_2_33 = Fraction(1, 1 << 20)  # results stay below 2^33: ulp at most 2^-20 (half of it, with room)
    for p in range(1, 1025):
        inv, c = constants(p)
        e_inv = abs(Fraction(inv) - Fraction(1, p))
        e_c = abs(Fraction(c) - Fraction(2 * p - 1, 2 * p))
        err = U_MAX * e_inv + e_c + half_ulp_at_2_33
        assert err < Fraction(1, 2 * p), p


def test_shortcut_exact_at_critical_work_amounts():
    rng = np.random.default_rng(2024)
    for p in range(1, 1025):
        kmax = (U_MAX - 2) // p
        ks = {0, 1, 2, 3, kmax, kmax - 1, max(kmax // 2, 0)}
        for m in range(10, 33):          # where the double's exponent steps
            k = (1 << m) // p
            ks.update({k - 1, k, k + 1})
        ks.update(int(v) for v in rng.integers(0, kmax + 1, size=12))
        for k in ks:
            if k < 0 or k > kmax:
                continue
            for u in (k * p - 1, k * p, k * p + 1):
                if 0 <= u < U_MAX:
                    assert shortcut(u, p) == -(-u // p), (u, p)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7, 850, 1016, 1023, 1024])
def test_shortcut_exhaustive_small_u(p):
    for u in range(0, 4 * p + 3):
        assert shortcut(u, p) == -(-u // p), (u, p)


def test_a_plain_reciprocal_would_fail():
    """The 1/2 offset matters: trunc(u * (1/p)) + 1 fails at exact multiples,
    and a ceiling of the rounded quotient fails where u/p rounds up past an
    integer; the shortcut's offset keeps 1/(2p) of room on both sides."""
    bad = 0
    for p in (3, 7, 11, 1000):
        for k in (1, 12345, (U_MAX - 2) // p):
            u = k * p
            if math.trunc(u * (1.0 / p)) + 1 != -(-u // p):
                bad += 1
    assert bad > 0
