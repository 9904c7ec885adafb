"""Exact master-equation pins on the 4x4 torus (CPU only).

The enumerator (oracle/enum4x4.py) works on heights and is independent of
the C oracle.  It is itself pinned by two independent state enumerations,
stochasticity, the flat-state width 1/4 (Sec. III) and, for p = q, the
closed-form stationary law: Eq. (1) with p = q is symmetric, so the chain is
doubly stochastic and its stationary law is uniform over all states.  The C
oracle's Monte Carlo histograms of W^2(t) (tiled dynamics and
random-sequential reference) must then match the exact laws.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import enum4x4 as E


def test_state_space_two_ways():
    a = E.states()
    b = E.states_by_slopes()
    assert a == b
    assert len(a) == 990


def test_flat_state_and_width_range():
    flat = E.states()[E.flat_index()]
    assert E.w2_exact(flat) == Fraction(1, 4)
    ws = [E.w2_exact(s) for s in E.states()]
    assert min(ws) == Fraction(1, 4)
    # C oracle flat state is the same configuration
    lat = oracle.flat(4, 4)
    bx = tuple(int(v) for v in (lat & 1).ravel())
    by = tuple(int(v) for v in ((lat >> 1) & 1).ravel())
    assert bx + by == flat


@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.95, 0.05), (0.5, 0.5)])
def test_chains_are_stochastic(p, q):
    for M in (E.rsu_mcs_matrix(p, q), E.tiled_mcs_matrix(p, q)):
        assert np.allclose(M.sum(axis=1), 1.0, atol=1e-12)
        assert M.min() >= -1e-15


def test_symmetric_rates_give_uniform_stationary_law():
    mean_uniform = sum(E.w2_exact(s) for s in E.states()) / len(E.states())
    assert mean_uniform == Fraction(92, 165)
    for M in (E.rsu_mcs_matrix(0.5, 0.5), E.tiled_mcs_matrix(0.5, 0.5)):
        assert np.allclose(M, M.T, atol=1e-12)  # symmetric => doubly stochastic
        pi = E.evolve(M, [400])[400]
        assert np.allclose(pi, 1.0 / 990, atol=1e-9)
        assert abs(E.mean_w2(pi) - 92 / 165) < 1e-9


def test_draw_probabilities_sum_and_balance():
    P = E.draw_probabilities(4)
    assert abs(P.sum() - 1) < 1e-15
    assert np.all(np.abs(P * 9 - 1) < 2e-4)  # 16-bit draw: near-uniform over 9 sites


def _histogram_test(S1S2, law, N=16):
    """Chi-square of the W^2 histogram of an ensemble against an exact law."""
    num = N * S1S2[:, 1] - S1S2[:, 0] ** 2
    keys = sorted(law)
    want = np.array([law[k] for k in keys]) * len(num)
    got = np.array([np.sum(num * k.denominator == k.numerator * N * N) for k in keys])
    assert got.sum() == len(num), "every sampled W^2 must be one of the exact values"
    keep = want >= 5
    obs = np.append(got[keep], got[~keep].sum())
    exp = np.append(want[keep], want[~keep].sum())
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    exp = exp * obs.sum() / exp.sum()
    return stats.chisquare(obs, exp).pvalue


@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.95, 0.05), (0.5, 0.5)])
@pytest.mark.parametrize("rsu", [False, True])
def test_oracle_histograms_match_exact_law(p, q, rsu):
    R, tmax = 40000, 10
    ens = oracle.ensemble(4, 4, p, q, seed0=1000, R=R, tmax=tmax, rsu=rsu)
    M = E.rsu_mcs_matrix(p, q) if rsu else E.tiled_mcs_matrix(p, q)
    laws = E.evolve(M, [1, 2, 10])
    for t in (1, 2, 10):
        pv = _histogram_test(ens[:, t - 1, :], E.w2_law(laws[t]))
        assert pv > 1e-4, f"t={t}: p-value {pv}"
        mean = np.mean((16 * ens[:, t - 1, 1] - ens[:, t - 1, 0] ** 2) / 256.0)
        assert abs(mean - E.mean_w2(laws[t])) < 5 * 0.2 / np.sqrt(R)


def test_tiled_and_rsu_laws_differ_at_small_size():
    """Sanity of the test's power: at L = 4 the dead rows change the law, and
    the histogram test tells the two chains apart."""
    R = 40000
    ens = oracle.ensemble(4, 4, 1.0, 0.0, seed0=5, R=R, tmax=1, rsu=False)
    rsu_law = E.w2_law(E.evolve(E.rsu_mcs_matrix(1.0, 0.0), [1])[1])
    assert _histogram_test(ens[:, 0, :], rsu_law) < 1e-6


# Mean W^2 of the random-sequential chain on the 4x4 torus from the flat
# state, at t = 1, 2, 10 MCS and in the stationary state, as found by a
# separate enumeration of the same master equation written independently of
# this package (its t = 1 value for p = 1 was also checked by a Monte Carlo
# run: 0.49448 +- 0.00038).  Six digits; the p = q stationary value is the
# closed form 92/165 of the uniform law.
I9_RSU_MEAN_W2 = {
    (1.0, 0.0): (0.494399, 0.545255, 0.583881, 0.583896),
    (0.95, 0.05): (0.500674, 0.543048, 0.580712, 0.580730),
    (0.5, 0.5): (0.529193, 0.549880, 0.557547, 92 / 165),
}


@pytest.mark.parametrize("pq", sorted(I9_RSU_MEAN_W2))
def test_random_sequential_law_matches_fixed_values(pq):
    """Fixed values pin the enumerator at p != q, where no closed form holds:
    a wrong rate, a transposed matrix or a wrong attempt count per MCS moves
    these means far beyond the sixth digit."""
    want = I9_RSU_MEAN_W2[pq]
    M = E.rsu_mcs_matrix(*pq)
    laws = E.evolve(M, [1, 2, 10])
    got = [E.mean_w2(laws[t]) for t in (1, 2, 10)]
    # stationary law: the left eigenvector of eigenvalue 1
    w, v = np.linalg.eig(M.T)
    pi = np.real(v[:, np.argmin(np.abs(w - 1.0))])
    pi = pi / pi.sum()
    got.append(E.mean_w2(pi))
    for g, x in zip(got, want):
        assert abs(g - x) < 1e-6, (pq, got, want)
