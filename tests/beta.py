"""Effective growth exponent of Sec. III, Eq. (beff), with jackknife errors.

beta_eff(t) = [ln W(t) - ln W(t')] / [ln t - ln t'] with t/t' = 2, where W^2 is
the ensemble mean of the excess width W^2 - 1/4 (the flat state's intrinsic
width 1/4 is subtracted first, Sec. III).  Realizations (seeds) are the
independent samples; errors and covariances come from the delete-one
jackknife over them.  Test-side statistics only: no part of the dynamics.
"""
import numpy as np


def excess_w2(S1, S2, N):
    """W^2 - 1/4 per sample from exact sums (numerator in Python integers)."""
    S1 = np.asarray(S1, dtype=object)
    S2 = np.asarray(S2, dtype=object)
    num = N * S2 - S1 * S1
    return np.array(num / (N * N), dtype=float) - 0.25


def pick_times(available, targets):
    """The available measurement time nearest to each target time."""
    a = np.asarray(available)
    return [int(a[np.argmin(np.abs(a - t))]) for t in targets]


def beta_eff(mean_w2, times):
    """beta_eff between consecutive times from ensemble-mean excess W^2."""
    lw = 0.5 * np.log(np.asarray(mean_w2, dtype=float))
    lt = np.log(np.asarray(times, dtype=float))
    return (lw[1:] - lw[:-1]) / (lt[1:] - lt[:-1])


def jackknife(w2, times):
    """w2: (R, T) excess widths of R realizations at T times.  Returns
    (beta, cov): beta_eff from the full ensemble and the jackknife covariance
    matrix of its T - 1 values."""
    w2 = np.asarray(w2, dtype=float)
    R = w2.shape[0]
    full = beta_eff(w2.mean(axis=0), times)
    tot = w2.sum(axis=0)
    loo = np.array([beta_eff((tot - w2[r]) / (R - 1), times) for r in range(R)])
    d = loo - loo.mean(axis=0)
    cov = (R - 1) / R * d.T @ d
    return full, cov
