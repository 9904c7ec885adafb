"""Pins of the beta_eff statistics (tests/beta.py) on closed forms (CPU)."""
import numpy as np

from tests import beta as B


def test_pure_power_law_gives_its_exponent():
    t = np.array([64, 128, 256, 512, 1024])
    for b in (0.1, 0.2415, 0.25, 1 / 3):
        w2 = 3.7 * t ** (2 * b)
        assert np.allclose(B.beta_eff(w2, t), b, atol=1e-12)
    # uneven ratios: the log difference is exact, not a ratio-of-2 shortcut
    t2 = np.array([60, 131, 250])
    assert np.allclose(B.beta_eff(2.0 * t2 ** 0.5, t2), 0.25, atol=1e-12)


def test_jackknife_of_identical_realizations_has_no_spread():
    t = np.array([100, 200, 400])
    w2 = np.tile(t ** 0.48, (10, 1))
    beta, cov = B.jackknife(w2, t)
    assert np.allclose(beta, 0.24) and np.allclose(cov, 0)


def test_jackknife_error_of_a_linear_estimator_is_the_standard_error():
    # for two times, ln of the means is nonlinear; but with w2 at t' fixed
    # and small relative spread at t, the jackknife variance of
    # 0.5 ln(mean) / ln 2 approaches (s / mean)^2 / R / (2 ln 2)^2
    rng = np.random.default_rng(4)
    R = 400
    a = 1 + 1e-3 * rng.standard_normal(R)
    w2 = np.stack([np.ones(R), a], axis=1)
    _, cov = B.jackknife(w2, np.array([1, 2]))
    want = a.var(ddof=1) / a.mean() ** 2 / R / (2 * np.log(2)) ** 2
    assert abs(cov[0, 0] / want - 1) < 1e-2


def test_excess_width_is_exact_for_large_sums():
    N = 2**34
    # flat state: S1 = S2 = N/2 gives exactly zero excess
    assert B.excess_w2([N // 2], [N // 2], N)[0] == 0.0
    # a surface of height H everywhere plus the zig-zag: excess 0 for any H
    H = 10**6
    S1 = N * H + N // 2
    S2 = N * H * H + 2 * H * (N // 2) + N // 2
    assert B.excess_w2([S1], [S2], N)[0] == 0.0


def test_pick_times():
    assert B.pick_times([11, 21, 62, 130, 250], [64, 128, 256]) == [62, 130, 250]
