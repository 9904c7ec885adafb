"""Steady-state width statistics of Sec. IV -- TEST INFRASTRUCTURE ONLY.

Written out from their definitions in exact rational arithmetic
(``fractions.Fraction``), for checking the library's statistics:

* W^2 of one sample from the exact sums, Eq. (Wdef): (N S2 - S1^2) / N^2;
* the non-central moments nu_n = <(W^2)^n> of a set of samples and the
  cumulants kappa_1..kappa_4 obtained from them as in Eq. (cumulants);
* the scaled distribution Psi_L(x) = <W^2> P_L(W^2 / <W^2>), estimated as
  the density of x = W^2 / <W^2> on equal bins.

Only ``tests/`` may import this module; it imports nothing from the HIP
library.
"""
from __future__ import annotations

from fractions import Fraction


def w2_exact(S1: int, S2: int, N: int) -> Fraction:
    """W^2 = S2/N - (S1/N)^2 of one sample, exactly (Eq. (Wdef))."""
    return Fraction(N * S2 - S1 * S1, N * N)


def moments(values) -> list:
    """[nu_1, nu_2, nu_3, nu_4]: the averages of v, v^2, v^3, v^4."""
    vals = [Fraction(v) for v in values]
    if not vals:
        raise ValueError("no samples")
    M = len(vals)
    return [sum(v ** n for v in vals) / M for n in (1, 2, 3, 4)]


def cumulants(values) -> list:
    """[kappa_1, ..., kappa_4] from the non-central moments (Eq. (cumulants))."""
    n1, n2, n3, n4 = moments(values)
    return [n1,
            n2 - n1 ** 2,
            n3 - 3 * n1 * n2 + 2 * n1 ** 3,
            n4 - 4 * n3 * n1 - 3 * n2 ** 2 + 12 * n1 ** 2 * n2 - 6 * n1 ** 4]


def psi(values, x_hi: float, nbins: int) -> list:
    """Density of x = v / <v> on nbins equal bins of [0, x_hi): bin i holds
    (samples with i dx <= x < (i+1) dx) / (M dx), dx = x_hi / nbins."""
    vals = [Fraction(v) for v in values]
    M = len(vals)
    mean = sum(vals) / M
    dx = Fraction(x_hi) / nbins
    counts = [0] * nbins
    for v in vals:
        k = (v / mean) // dx
        if 0 <= k < nbins:
            counts[int(k)] += 1
    return [float(c / (M * dx)) for c in counts]
