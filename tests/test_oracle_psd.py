"""Pins of the oracle's power spectrum (Eqs. (PSD), (hF)) to closed forms,
Parseval's identity against the exact width, symmetries of the surface and
a brute-force transform of tiny lattices."""
import cmath
import math

import numpy as np
import pytest

import oracle
from oracle import psd as P
from tests import inputs


def test_cosine_profiles_closed_form():
    # h = A cos(2 pi n0 x / Lx) + B cos(2 pi m0 y / Ly) has mean zero and
    # h(k) = A Lx Ly / (2 sqrt(Lx Ly)) at k = (2 pi n0 / Lx, 0): S = A^2 Lx Ly / 4,
    # and likewise B^2 Lx Ly / 4 at (0, 2 pi m0 / Ly); every other axis value is 0
    Lx, Ly, A, B, n0, m0 = 32, 16, 3.0, 5.0, 3, 2
    x = np.arange(Lx)[None, :]
    y = np.arange(Ly)[:, None]
    h = A * np.cos(2 * np.pi * n0 * x / Lx) + B * np.cos(2 * np.pi * m0 * y / Ly)
    Sx, Sy = P.psd_axes(h)
    assert Sx.shape == (Lx // 2 + 1,) and Sy.shape == (Ly // 2 + 1,)
    ex = np.zeros_like(Sx)
    ex[n0] = A * A * Lx * Ly / 4
    ey = np.zeros_like(Sy)
    ey[m0] = B * B * Lx * Ly / 4
    assert np.allclose(Sx, ex, atol=1e-9) and np.allclose(Sy, ey, atol=1e-9)


def test_nyquist_checkerboard_of_the_flat_state():
    # flat zig-zag h = (x + y) mod 2: h - <h> = (-1)^(x+y) / 2 lives on
    # k = (pi, pi) only, with S = N / 4 there; nothing on the axes
    lat = oracle.flat(16, 8)
    S = P.psd_full(oracle.heights(lat, 0))
    ex = np.zeros_like(S)
    ex[4, 8] = 16 * 8 / 4
    assert np.allclose(S, ex, atol=1e-12)
    Sx, Sy = P.psd(lat, 0)
    assert np.allclose(Sx, 0, atol=1e-12) and np.allclose(Sy, 0, atol=1e-12)


def test_square_wave_closed_form():
    # h = [x < Lx/2] on an Lx x Ly lattice: for odd n,
    # |sum_x h e^{-2 pi i n x / Lx}| = Ly / sin(pi n / Lx), so
    # S = Ly / (Lx sin^2(pi n / Lx)); even n > 0 give 0
    Lx, Ly = 16, 8
    h = np.zeros((Ly, Lx))
    h[:, : Lx // 2] = 1
    Sx, Sy = P.psd_axes(h)
    for n in range(1, Lx // 2 + 1):
        want = Ly / (Lx * math.sin(math.pi * n / Lx) ** 2) if n % 2 else 0.0
        assert abs(Sx[n] - want) < 1e-9, n
    assert np.allclose(Sy, 0, atol=1e-12)
    assert abs(Sx[0]) < 1e-12


@pytest.mark.parametrize("Lx,Ly,seed", [(32, 32, 1), (64, 32, 2), (32, 96, 3)])
def test_parseval_equals_exact_width(Lx, Ly, seed):
    # sum over the whole reciprocal lattice of S = sum (h - <h>)^2 = N W^2,
    # with W^2 from the exact integer sums of Eq. (Wdef)
    lat, H0 = inputs.rough_state(Lx, Ly, seed=seed, mcs=3)
    S = P.psd_full(oracle.heights(lat, H0))
    S1, S2 = oracle.width_sums(lat, H0)
    N = Lx * Ly
    assert abs(S.sum() - N * oracle.w2(S1, S2, N)) < 1e-9 * max(1.0, S.sum())


def test_translation_and_mirror_invariance():
    # shifting the surface or flipping h -> -h (complementing every slope
    # bit) leaves |h(k)|^2 unchanged
    lat, H0 = inputs.rough_state(64, 32, seed=7, mcs=4)
    Sx, Sy = P.psd(lat, H0)
    assert Sx[1:].max() > 0 and Sy[1:].max() > 0
    for dy, dx in [(0, 5), (3, 0), (11, 29)]:
        Rx, Ry = P.psd(np.roll(lat, (dy, dx), axis=(0, 1)), 17)
        assert np.allclose(Rx, Sx, rtol=1e-12, atol=1e-9)
        assert np.allclose(Ry, Sy, rtol=1e-12, atol=1e-9)
    Mx, My = P.psd(lat ^ 3, -H0)
    assert np.allclose(Mx, Sx, rtol=1e-12, atol=1e-9) and np.allclose(My, Sy, rtol=1e-12, atol=1e-9)


def test_brute_force_on_a_tiny_lattice():
    # direct double sum of Eq. (hF) along both axes, in Python complex numbers
    lat, H0 = inputs.rough_state(8, 8, seed=5, mcs=5)
    h = oracle.heights(lat, H0)
    Ly, Lx = h.shape
    mean = sum(int(v) for v in h.ravel()) / (Lx * Ly)
    Sx, Sy = P.psd(lat, H0)
    for n in range(Lx // 2 + 1):
        acc = sum((int(h[y, x]) - mean) * cmath.exp(2j * math.pi * n * x / Lx)
                  for y in range(Ly) for x in range(Lx)) / math.sqrt(Lx * Ly)
        assert abs(abs(acc) ** 2 - Sx[n]) < 1e-9
    for n in range(Ly // 2 + 1):
        acc = sum((int(h[y, x]) - mean) * cmath.exp(2j * math.pi * n * y / Ly)
                  for y in range(Ly) for x in range(Lx)) / math.sqrt(Lx * Ly)
        assert abs(abs(acc) ** 2 - Sy[n]) < 1e-9


def test_direction_average():
    a, b = np.arange(5.0), np.arange(5.0) * 3
    assert np.array_equal(P.direction_average(a, b), 2 * np.arange(5.0))
    with pytest.raises(ValueError):
        P.direction_average(np.zeros(3), np.zeros(4))
