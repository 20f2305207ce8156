"""Host-side calibration fits of the C ABI (tgo_fit_line, tgo_fit_overlap)
against their definitions: least squares (numpy's polyfit) and the
overlapped-transfer rates of the model (Section 4.2.1) recovered from
transfers simulated by the CPU oracle."""
import numpy as np
import pytest

from oracle import model as M


@pytest.fixture(scope="module")
def tgo():
    from paper_1806_10113_amd import tgo as t
    t.lib()
    return t


def test_fit_line_is_least_squares(tgo):
    rng = np.random.default_rng(70)
    for _ in range(50):
        n = int(rng.integers(2, 40))
        x = rng.uniform(0, 1e9, n)
        y = 3.7e-2 * x + 1.5e4 + rng.normal(0, 1e3, n)
        a, b = tgo.fit_line(x, y)
        ra, rb = np.polyfit(x, y, 1)
        assert a == pytest.approx(ra, rel=1e-9, abs=1e-15) and b == pytest.approx(rb, rel=1e-6, abs=1e-6)
    # points on a line are recovered exactly (Eq. 1: T = eta m + gamma)
    a, b = tgo.fit_line([1, 2, 3, 10], [7, 9, 11, 25])
    assert (a, b) == (2.0, 5.0)
    with pytest.raises(tgo.TgoError):
        tgo.fit_line([1.0, 1.0], [2.0, 3.0])


def overlap_times(h, d, delay, m):
    """An HtD of h and a DtH of d issued `delay` after it, simulated by the
    oracle: task 0 = (0, delay, d) holds its DtH back with a kernel of length
    delay; task 1 = (h, 0, 0) is the HtD."""
    T, ev = M.simulate([(0, delay, d), (h, 0, 0)], [0, 1], m, trace=True)
    Te = M.simulate([(0, delay, d), (h, 0, 0)], [0, 1], m, exact=True)
    hs, he = ev[("HtD", 1)]
    ds, de = ev[("DtH", 0)]
    return [hs, he, ds, de], T == Te


def test_fit_overlap_recovers_model_rates(tgo):
    rng = np.random.default_rng(71)
    for q, ph, pd in ((4, 3, 3), (4, 2, 2), (4, 3, 1), (8, 5, 7), (16, 9, 13)):
        m = M.Model(q, ph, pd)
        times, solo = [], []
        while len(times) < 6:
            h = int(rng.integers(1, 50)) * 720720
            d = int(rng.integers(1, 50)) * 720720
            delay = int(rng.integers(0, 2)) * int(rng.integers(0, h // 720720 + 1)) * 720720 // 2
            t, exact = overlap_times(h, d, delay, m)
            if not exact or min(t[1], t[3]) <= max(t[0], t[2]):
                continue  # keep experiments without rounding that overlap
            times.append(t)
            solo.append([h, d])
        rh, rd = tgo.fit_overlap(np.array(times), np.array(solo))
        assert rh == pytest.approx(ph / q, rel=1e-12) and rd == pytest.approx(pd / q, rel=1e-12)


def test_fit_overlap_skips_non_overlapping(tgo):
    m = M.Model(4, 3, 3)
    t_no, _ = overlap_times(1000, 1000, 5000, m)   # DtH starts after the HtD ends
    t_ov, _ = overlap_times(1200, 1200, 0, m)
    rh, rd = tgo.fit_overlap(np.array([t_no, t_ov]), np.array([[1000, 1000], [1200, 1200]]))
    assert rh == pytest.approx(0.75) and rd == pytest.approx(0.75)
    # no overlap at all: an argument error (the device validation then keeps
    # solo rates and reports that no overlap was observed)
    with pytest.raises(tgo.TgoError) as ei:
        tgo.fit_overlap(np.array([t_no]), np.array([[1000, 1000]]))
    assert ei.value.code == tgo.TGO_EINVAL
