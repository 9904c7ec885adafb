"""Pins of the oracle's steady-state statistics (Sec. IV, Eq. (cumulants)).

The cumulant formulas are checked against closed forms of distributions
whose cumulants are textbook results, against scipy's central moments, and
against the scaling and shift laws of cumulants; Psi against its
normalisation.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats as sst

from oracle import stats


@pytest.mark.parametrize("n", [1, 2, 5, 10, 37])
def test_discrete_uniform_closed_forms(n):
    # population cumulants of the uniform distribution on {1, ..., n}
    k = stats.cumulants(range(1, n + 1))
    assert k[0] == Fraction(n + 1, 2)
    assert k[1] == Fraction(n * n - 1, 12)
    assert k[2] == 0
    assert k[3] == -Fraction((n * n - 1) * (n * n + 1), 120)


@pytest.mark.parametrize("ones,total", [(1, 2), (1, 3), (3, 10), (7, 8)])
def test_two_point_closed_forms(ones, total):
    p = Fraction(ones, total)
    k = stats.cumulants([1] * ones + [0] * (total - ones))
    assert k == [p, p * (1 - p), p * (1 - p) * (1 - 2 * p), p * (1 - p) * (1 - 6 * p * (1 - p))]


def test_against_scipy_central_moments():
    rng = np.random.default_rng(3)
    x = rng.gamma(2.0, 1.5, size=2000)
    k = [float(v) for v in stats.cumulants(x.tolist())]
    m2, m3, m4 = (sst.moment(x, m) for m in (2, 3, 4))
    assert k[0] == pytest.approx(x.mean(), rel=1e-12)
    assert k[1] == pytest.approx(m2, rel=1e-12)
    assert k[2] == pytest.approx(m3, rel=1e-10)
    assert k[3] == pytest.approx(m4 - 3 * m2 * m2, rel=1e-10)


def test_shift_and_scale_laws():
    vals = [Fraction(v) for v in (3, 5, 5, 8, 13, 2, 9, 9, 9, 1)]
    k = stats.cumulants(vals)
    c, s = Fraction(7, 3), Fraction(-5, 2)
    ks = stats.cumulants([s * v + c for v in vals])
    assert ks[0] == s * k[0] + c
    for n in (2, 3, 4):
        assert ks[n - 1] == s ** n * k[n - 1]


def test_w2_of_flat_state_is_a_quarter():
    for L in (4, 32, 1024):
        N = L * L
        assert stats.w2_exact(N // 2, N // 2, N) == Fraction(1, 4)


def test_psi_normalisation():
    rng = np.random.default_rng(5)
    vals = (rng.gamma(3.0, 1.0, size=500) + 0.1).tolist()
    mean = sum(Fraction(v) for v in vals) / len(vals)
    x_hi, nb = 3.0, 30
    p = stats.psi(vals, x_hi, nb)
    inside = sum(1 for v in vals if Fraction(v) / mean < Fraction(x_hi))
    assert sum(p) * (x_hi / nb) == pytest.approx(inside / len(vals), rel=1e-12)
    # all mass on one value: the density is 1/dx in the bin holding x = 1
    p1 = stats.psi([2.5] * 7, 2.0, 4)
    assert p1 == [0.0, 0.0, 2.0, 0.0]
