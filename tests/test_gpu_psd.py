"""GPU power spectrum (Eqs. (PSD), (hF)) against the oracle's fft2 of the
reconstructed heights, on oracle-made surfaces, up to the paper's L = 2^13.

Tolerance (fp64 radix-2 FFT, Higham, Accuracy and Stability, Thm. 24.2): a
length-n transform of x has ||dZ||_2 <= (7 log2 n + 1) u sqrt(n) ||x||_2 with
u = 2^-53, the +1 covering the rounding of the mean-subtracted input.  The
library transforms the column (row) profile of length Lx (Ly); the oracle
transforms all N = Lx Ly heights.  With delta the sum of the two bounds and
Z = sqrt(N S) the oracle's coefficient, |S_gpu - S_oracle| <= (2 |Z| + delta) delta / N.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import psd as P
from tests import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def okpz():
    from paper_1110_6745_amd import okpz as m

    return m


def fft_bound(n, norm2):
    if n & (n - 1) == 0:
        return (7 * math.log2(n) + 1) * U * math.sqrt(n) * norm2
    # Bluestein: a = x c and the chirp b (2n - 1 unit entries) through two
    # length-M transforms, a product bounded by |B^| <= 2n and |A^| <= ||a||_1,
    # and the undone transform: ||dX||_2 <= 5.5 n gamma_M ||x||_2, taken as 6
    M = 1
    while M < 2 * n - 1:
        M *= 2
    return 6 * n * (7 * math.log2(M) + 1) * U * norm2


def check(got, lat, H0, what):
    h = oracle.heights(lat, H0)
    Ly, Lx = h.shape
    N = Lx * Ly
    Sx, Sy = P.psd_axes(h)
    hc = h - h.mean()
    d_or = fft_bound(N, float(np.linalg.norm(hc)))
    for axis, S_gpu, S_or, prof in ((0, got[0], Sx, h.sum(axis=0)), (1, got[1], Sy, h.sum(axis=1))):
        n = prof.size
        assert S_gpu.shape == S_or.shape, what
        delta = d_or + fft_bound(n, float(np.linalg.norm(prof - prof.mean())))
        tol = (2 * np.sqrt(N * np.maximum(S_or, 0)) + delta) * delta / N
        assert S_gpu[0] == 0.0, what
        bad = np.abs(S_gpu - S_or) > tol
        assert not bad.any(), (f"{what} axis {axis}: n={np.flatnonzero(bad)[:5]} "
                               f"gpu={S_gpu[bad][:3]} oracle={S_or[bad][:3]} tol={tol[bad][:3]}")


@pytest.mark.parametrize("Lx,Ly", [(32, 32), (64, 128), (4096, 32), (32, 2048)])
def test_flat_state_has_an_empty_axis_spectrum(okpz, Lx, Ly):
    sim = okpz.okpz_init(Lx, Ly, 1.0, 0.0, 1)
    sx, sy = sim.psd()
    assert sx.shape == (Lx // 2 + 1,) and sy.shape == (Ly // 2 + 1,)
    assert not sx.any() and not sy.any()
    sim.free()


@pytest.mark.parametrize("Lx,Ly,seed", [(32, 32, 1), (64, 128, 2), (128, 64, 3), (256, 256, 4),
                                        (1024, 512, 5), (2048, 2048, 6), (8192, 32, 7),
                                        (131072, 32, 8), (32, 131072, 9)])
def test_rough_surfaces_match_oracle(okpz, Lx, Ly, seed):
    lat, H0 = inputs.rough_state(Lx, Ly, seed=seed, mcs=4)
    sim = okpz.okpz_init(Lx, Ly, 0.9, 0.2, seed)
    sim.set_lattice(lat, H0, 100)
    check(sim.psd(), lat, H0, f"{Lx}x{Ly} as loaded")
    # after sweeps the stored columns are rotated (block shift); the oracle
    # evolves its own copy
    Hr = H0
    for s in range(100, 103):
        Hr = oracle.sweep(lat, 0.9, 0.2, seed, s, Hr)
    sim.sweep(3)
    check(sim.psd(), lat, Hr, f"{Lx}x{Ly} after 3 sweeps")
    sim.free()


def test_paper_scale_lattice(okpz):
    # the paper's spectrum is taken on L = 2^13 (Sec. III)
    L = 8192
    lat, H0 = inputs.rough_state(L, L, seed=11, mcs=1)
    sim = okpz.okpz_init(L, L, 1.0, 0.0, 11)
    sim.set_lattice(lat, H0, 0)
    Hr = H0
    for s in range(2):
        Hr = oracle.sweep(lat, 1.0, 0.0, 11, s, Hr)
    sim.sweep(2)
    check(sim.psd(), lat, Hr, "8192^2")
    sim.free()


def test_growth_from_flat_matches_oracle_and_repeats(okpz):
    L = 512
    sim = okpz.okpz_init(L, L, 1.0, 0.0, 3)
    lat, H = oracle.flat(L, L), 0
    H = oracle.run(lat, 1.0, 0.0, 3, 0, 20, H)
    sim.sweep(20)
    a = sim.psd()
    check(a, lat, H, "512^2 growth t=20")
    b = sim.psd()  # scratch reused: same answer
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    sim.free()


@pytest.mark.parametrize("Lx,Ly,seed", [(96, 64, 21), (64, 96, 22), (96, 96, 23), (320, 192, 24),
                                        (1056, 96, 25), (3072, 2080, 26)])
def test_sides_that_are_not_powers_of_two(okpz, Lx, Ly, seed):
    # Bluestein's chirp-z transform on such sides (either or both)
    lat, H0 = inputs.rough_state(Lx, Ly, seed=seed, mcs=4)
    sim = okpz.okpz_init(Lx, Ly, 0.95, 0.05, seed)
    sim.set_lattice(lat, H0, 0)
    check(sim.psd(), lat, H0, f"{Lx}x{Ly} as loaded")
    sim.sweep(2)
    Hr = oracle.run(lat, 0.95, 0.05, seed, 0, 2, H0)
    check(sim.psd(), lat, Hr, f"{Lx}x{Ly} after 2 sweeps")
    sim.free()
