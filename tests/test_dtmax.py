"""CPU tests of the time-step decision rules (Sec. V.B, Table 1) on synthetic
curves with known decay constants."""
import numpy as np
import pytest

from paper_1411_3487_amd import dtmax

TS = 100.0
K = 14
LAGS = np.array([0.0] + [TS * 2 ** (j - 1) for j in range(1, K)])
NAMES = ("L", "umid", "msd")


def curves(rates, amp=(3.0, 1.0, 2.0)):
    """Two exponential autocorrelations and an msd 2(1 - e^{-r t}), with
    decay constants rates = (r_L, r_u, r_msd)."""
    q = np.zeros((K, 3))
    q[:, 0] = amp[0] * np.exp(-rates[0] * LAGS)
    q[:, 1] = amp[1] * np.exp(-rates[1] * LAGS)
    q[:, 2] = amp[2] * (1 - np.exp(-rates[2] * LAGS))
    return q


def test_decay_constant_of_an_exponential_is_exact():
    r = 1.3e-4
    q = 2.0 * np.exp(-r * LAGS)
    for t in (100, 1e3, 1e4, 1e5):
        val, lag = dtmax.decay_constant(q, LAGS, t)
        assert val == pytest.approx(-r, rel=1e-12)
        assert lag == LAGS[np.argmin(np.abs(LAGS - t))]


def test_decay_constant_of_two_exponentials_matches_the_derivative():
    """Central difference of ln Q over neighbouring lags against the analytic
    d ln Q / d tau, within the difference's error for this smooth curve."""
    a, b = 1e-3, 1e-5
    q = np.exp(-a * LAGS) + 4 * np.exp(-b * LAGS)
    val, lag = dtmax.decay_constant(q, LAGS, 1e4)
    dq = -a * np.exp(-a * lag) - 4 * b * np.exp(-b * lag)
    exact = dq / (np.exp(-a * lag) + 4 * np.exp(-b * lag))
    assert val == pytest.approx(exact, rel=0.3)
    assert val < 0


def test_decay_constant_needs_positive_neighbours():
    q = np.ones(K)
    q[5] = -1.0
    assert dtmax.decay_constant(q, LAGS, LAGS[4])[0] is None


def test_qt_ratios_within_and_outside_the_ten_percent_band():
    base = (2e-5, 1e-4, 3e-4)
    ref = curves(base)
    close = curves([r * 1.05 for r in base])
    far = curves([base[0], base[1] * 1.15, base[2]])
    r_ok, ok = dtmax.qt_ratios(close, ref, LAGS, [1e3, 1e4], NAMES)
    assert ok and r_ok
    assert all(abs(v - 1.05) < 0.02 for k, v in r_ok.items() if not k.startswith("msd"))
    r_bad, bad = dtmax.qt_ratios(far, ref, LAGS, [1e3, 1e4], NAMES)
    assert not bad
    assert any(k.startswith("umid") and abs(v - 1.15) < 0.01 for k, v in r_bad.items())


def test_decayed_autocorrelations_are_skipped_but_msd_is_not():
    ref = curves((1e-2, 1e-2, 1e-2))         # decayed by lag ~300
    other = curves((5e-2, 5e-2, 5e-2))
    ratios, ok = dtmax.qt_ratios(other, ref, LAGS, [1e4], NAMES)
    assert not any(k.startswith(("L@", "umid@")) for k in ratios)
    assert ok  # the msd has saturated: both decay constants ~0 -> skipped or equal
    ratios, ok = dtmax.qt_ratios(other, ref, LAGS, [200], NAMES)
    assert "msd@200" in ratios and not ok


def test_q0_passes_the_five_percent_band():
    assert dtmax.q0_passes([1.0, 0.951, 1.049])
    assert not dtmax.q0_passes([1.0, 0.94, 1.0])
    assert not dtmax.q0_passes([1.06])


def test_contiguous_dtau_max():
    assert dtmax.contiguous_dtau_max([10, 50, 100, 200], [True, True, False, True]) == 50
    assert dtmax.contiguous_dtau_max([200, 10, 100, 50], [True, True, False, True]) == 50
    assert dtmax.contiguous_dtau_max([10, 50], [False, True]) is None
    assert dtmax.contiguous_dtau_max([10, 50], [True, True]) == 50
    assert dtmax.contiguous_dtau_max([], []) is None


def test_table_one_rows_from_synthetic_runs():
    """Whole decision chain: time steps whose decay constants drift by 0, 3,
    8 and 20 % from the reference give the largest step with drift <= 10 %,
    and the final value is the smaller of the two groups (Table 1's rule).
    The msd grows over the test times (r t <= 0.1), so its decay constant
    follows 1/t and barely depends on r."""
    base = (2e-6, 5e-5, 1e-6)
    ref = curves(base)
    dts = [1, 10, 100, 200, 500]
    drift = {10: 0.0, 100: 0.03, 200: 0.08, 500: 0.20}
    passes = [True]
    for dt in dts[1:]:
        c = curves([r * (1 + drift[dt]) for r in base])
        passes.append(dtmax.qt_ratios(c, ref, LAGS, [1e3, 1e4, 1e5], NAMES)[1])
    dyn = dtmax.contiguous_dtau_max(dts, passes)
    assert dyn == 200
    eq = dtmax.contiguous_dtau_max(dts, [dtmax.q0_passes([1 + 0.0002 * d]) for d in dts])
    assert eq == 200
    eq = dtmax.contiguous_dtau_max(dts, [dtmax.q0_passes([1 + 0.0004 * d]) for d in dts])
    assert eq == 100
    assert min(eq, dyn) == 100
