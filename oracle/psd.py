"""Power spectrum density of the surface, Eqs. (PSD) and (hF) of Sec. III --
TEST INFRASTRUCTURE ONLY.

Written out from the definition: the heights of the lattice (Sec. I
reconstruction, ``oracle.heights``), minus their mean, are Fourier
transformed over both lattice directions with the normalisation
1 / L^{d/2} of Eq. (hF), d = 2 (for an Lx x Ly lattice: 1 / sqrt(Lx Ly)), and
S(k) = h(k) h(-k) = |h(k)|^2 for one surface (h is real).  The library's
spectrum is the one along the two lattice axes, k = (2 pi n / Lx, 0) and
k = (0, 2 pi n / Ly), n = 0 .. L/2; its "average over the x and y
directions" is the mean of the two on a square lattice.  The ensemble
average <...> of Eq. (PSD) is a mean over realisations, taken by the caller.

numpy's FFT is the only library step.  Only ``tests/`` may import this
module; it imports nothing from the HIP library.
"""
from __future__ import annotations

import numpy as np


def psd_full(h: np.ndarray) -> np.ndarray:
    """S(k) on the whole reciprocal lattice of a height array of shape
    (Ly, Lx): entry [ny, nx] belongs to k = (2 pi nx / Lx, 2 pi ny / Ly).

    The exponent's sign in Eq. (hF) does not matter: h is real, so
    |h(k)| = |h(-k)|."""
    h = np.asarray(h, dtype=np.float64)
    Ly, Lx = h.shape
    hk = np.fft.fft2(h - h.mean()) / np.sqrt(Lx * Ly)
    return (hk * np.conj(hk)).real


def psd_axes(h: np.ndarray) -> tuple:
    """(Sx, Sy): S along the x axis for n = 0 .. Lx/2 and along the y axis
    for n = 0 .. Ly/2, from ``psd_full``."""
    S = psd_full(h)
    Ly, Lx = S.shape
    return S[0, : Lx // 2 + 1].copy(), S[: Ly // 2 + 1, 0].copy()


def psd(lat: np.ndarray, H0: int) -> tuple:
    """(Sx, Sy) of a lattice state (slope bytes as in ``oracle``) with
    height H0 at site (0,0)."""
    import oracle

    return psd_axes(oracle.heights(lat, H0))


def direction_average(Sx: np.ndarray, Sy: np.ndarray) -> np.ndarray:
    """The spectrum averaged over the x and y directions (square lattices)."""
    if Sx.shape != Sy.shape:
        raise ValueError("direction average needs a square lattice")
    return 0.5 * (Sx + Sy)
