"""okpz oracle -- TEST INFRASTRUCTURE ONLY.

Plain CPU reference of the octahedron-model hot path (Kelling & Odor,
arXiv:1110.6745): the seeded tiled dynamics of Sec. II, the textbook
random-sequential reference, height reconstruction (Sec. I) and the exact width
sums of Eq. (Wdef).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_1110_6745_amd``) and never imports it.

Lattice arrays are ``numpy.uint8`` of shape ``(Ly, Lx)``; bit 0 of a byte is
``bx = [sigma_x = +1]`` and bit 1 is ``by = [sigma_y = +1]`` of that site.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "okpz_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build() -> str:
    """Compile the oracle's C source into ``oracle/liboracle.so``."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-shared", "-fPIC", _SRC,
           "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    L = ctypes.CDLL(_LIB_PATH)
    L.or_philox.argtypes = [_u32p, _u32p, _u32p]
    L.or_philox.restype = None
    L.or_threshold.argtypes = [ctypes.c_double]
    L.or_threshold.restype = ctypes.c_uint64
    L.or_geometry.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32p, _i32p, _i32p]
    L.or_geometry.restype = ctypes.c_int
    L.or_flat.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int64]
    L.or_flat.restype = None
    L.or_block_sweep.argtypes = [_u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                 ctypes.c_int32, _i64p, _i64p, _i64p, _u8p, ctypes.c_int]
    L.or_block_sweep.restype = ctypes.c_int
    L.or_block_shift.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                 ctypes.c_int32, _i32p, _i32p]
    L.or_block_shift.restype = None
    L.or_sweep.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                           ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _i64p,
                           _i64p, _i64p, ctypes.c_int, ctypes.c_int]
    L.or_sweep.restype = ctypes.c_int
    L.or_rsu_sweep.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                               ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _i64p,
                               _i64p, _i64p]
    L.or_rsu_sweep.restype = None
    L.or_heights.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i64p]
    L.or_heights.restype = None
    L.or_width.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i64p,
                           _i64p]
    L.or_width.restype = ctypes.c_int
    L.or_ensemble.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                              ctypes.c_double, ctypes.c_uint64, ctypes.c_int64,
                              ctypes.c_int64, ctypes.c_int, _i64p]
    L.or_ensemble.restype = ctypes.c_int
    L.or_ensemble_at.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, _i64p,
                                 ctypes.c_int64, ctypes.c_int, _i64p]
    L.or_ensemble_at.restype = ctypes.c_int
    L.or_window_sweep.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_uint32, _i64p, _i64p, _i64p, _i64p, _i64p,
                                  ctypes.c_int]
    L.or_window_sweep.restype = ctypes.c_int
    L.or_width_rows.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_uint64), _i64p,
                                ctypes.POINTER(ctypes.c_uint64), _i64p, _i64p]
    L.or_width_rows.restype = None
    L.or_num_threads.argtypes = []
    L.or_num_threads.restype = ctypes.c_int
    L.or_set_num_threads.argtypes = [ctypes.c_int]
    L.or_set_num_threads.restype = None
    _lib = L
    return L


def _ptr(a: np.ndarray, t):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


def _check_lattice(lat: np.ndarray) -> None:
    if lat.dtype != np.uint8 or lat.ndim != 2 or not lat.flags["C_CONTIGUOUS"]:
        raise TypeError("lattice must be a C-contiguous uint8 array of shape (Ly, Lx)")


# --------------------------------------------------------------------------
# Random numbers and constants of the dynamics
# --------------------------------------------------------------------------
def philox(counter, key) -> tuple:
    """Philox4x32-10 of a 4-word counter under a 2-word key (Salmon et al.)."""
    c = np.asarray(counter, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(o, _u32p))
    return tuple(int(v) for v in o)


def threshold(prob: float) -> int:
    """Integer acceptance threshold T with accept iff draw < T (Eq. (1))."""
    return int(lib().or_threshold(float(prob)))


def geometry(Lx: int, Ly: int) -> tuple:
    """(Bx, By, C): block sides and thread-cell side of the decomposition."""
    bx, by, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    if lib().or_geometry(Lx, Ly, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(c)) != 0:
        raise ValueError(f"unsupported lattice {Lx}x{Ly}")
    return bx.value, by.value, c.value


def block_shift(seed: int, s: int, Bx: int, By: int) -> tuple:
    sx, sy = ctypes.c_int32(), ctypes.c_int32()
    lib().or_block_shift(seed, s, Bx, By, ctypes.byref(sx), ctypes.byref(sy))
    return sx.value, sy.value


# --------------------------------------------------------------------------
# Lattice states and dynamics
# --------------------------------------------------------------------------
def flat(Lx: int, Ly: int) -> np.ndarray:
    """Flat zig-zag initial state (Sec. III); its height at (0,0) is 0."""
    lat = np.empty((Ly, Lx), dtype=np.uint8)
    lib().or_flat(_ptr(lat, _u8p), Lx, Ly)
    return lat


class Counts:
    """Accepted attachments and detachments of a run."""

    def __init__(self):
        self.att = 0
        self.det = 0


def sweep(lat: np.ndarray, p: float, q: float, seed: int, s: int, H0: int,
          check: bool = False, counts: Counts | None = None, delayed: bool = False) -> int:
    """One MCS (sweep index ``s``) of the tiled dynamics, in place.

    Returns the new absolute height of site (0,0).  ``check`` turns on the
    bond-conflict checker (raises if any bond is touched twice in one step,
    or in one phase of a step with ``delayed``).  ``delayed`` selects the
    delayed thread-cell borders of Sec. II (bulk, then edge, then corner
    attempts of every step) instead of dead ones.
    """
    _check_lattice(lat)
    Ly, Lx = lat.shape
    h = ctypes.c_int64(H0)
    a, d = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib().or_sweep(_ptr(lat, _u8p), Lx, Ly, threshold(p), threshold(q), seed, s,
                        ctypes.byref(h), ctypes.byref(a), ctypes.byref(d), int(check),
                        int(delayed))
    if rc == -1:
        raise AssertionError("bond conflict inside one step of the tiled schedule")
    if rc != 0:
        raise ValueError(f"or_sweep failed ({rc})")
    if counts is not None:
        counts.att += a.value
        counts.det += d.value
    return h.value


def run(lat: np.ndarray, p: float, q: float, seed: int, t0: int, n: int, H0: int,
        check: bool = False, counts: Counts | None = None, delayed: bool = False) -> int:
    """Sweeps ``t0 .. t0+n-1`` of the tiled dynamics; returns the new H0."""
    for s in range(t0, t0 + n):
        H0 = sweep(lat, p, q, seed, s, H0, check=check, counts=counts, delayed=delayed)
    return H0


def block_sweep(blk: np.ndarray, C: int, seed: int, s: int, block_id: int, p: float,
                q: float, site00=(-1, -1), check: bool = False, delayed: bool = False) -> tuple:
    """One sweep of a single device-level block given as its (By, Bx) cut-out.

    Returns (dh00, n_att, n_det).  Blocks are independent within a sweep, so
    this reproduces the tiled sweep of any block of any lattice size.
    """
    _check_lattice(blk)
    By, Bx = blk.shape
    dh, a, d = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    touched = np.zeros(2 * Bx * By, dtype=np.uint8) if check else None
    rc = lib().or_block_sweep(_ptr(blk, _u8p), Bx, By, C, seed, s, block_id,
                              threshold(p), threshold(q), site00[0], site00[1],
                              ctypes.byref(dh), ctypes.byref(a), ctypes.byref(d),
                              _ptr(touched, _u8p) if check else None, int(delayed))
    if rc == -2:
        raise ValueError("delayed cell borders need a cell side of at least 2")
    if rc != 0:
        raise AssertionError("bond conflict inside one step of the tiled schedule")
    return dh.value, a.value, d.value


def rsu_sweep(lat: np.ndarray, p: float, q: float, seed: int, t: int, H0: int,
              counts: Counts | None = None) -> int:
    """One MCS (N attempts) of the random-sequential reference; returns new H0."""
    _check_lattice(lat)
    Ly, Lx = lat.shape
    h = ctypes.c_int64(H0)
    a, d = ctypes.c_int64(0), ctypes.c_int64(0)
    lib().or_rsu_sweep(_ptr(lat, _u8p), Lx, Ly, threshold(p), threshold(q), seed, t,
                       ctypes.byref(h), ctypes.byref(a), ctypes.byref(d))
    if counts is not None:
        counts.att += a.value
        counts.det += d.value
    return h.value


def rsu_run(lat, p, q, seed, t0, n, H0, counts=None) -> int:
    for t in range(t0, t0 + n):
        H0 = rsu_sweep(lat, p, q, seed, t, H0, counts=counts)
    return H0


# --------------------------------------------------------------------------
# Heights and width
# --------------------------------------------------------------------------
def heights(lat: np.ndarray, H0: int) -> np.ndarray:
    _check_lattice(lat)
    Ly, Lx = lat.shape
    h = np.empty((Ly, Lx), dtype=np.int64)
    lib().or_heights(_ptr(lat, _u8p), Lx, Ly, H0, _ptr(h, _i64p))
    return h


def width_sums(lat: np.ndarray, H0: int) -> tuple:
    """(S1, S2) = (sum h, sum h^2), exact; raises OverflowError past int64."""
    _check_lattice(lat)
    Ly, Lx = lat.shape
    s1, s2 = ctypes.c_int64(), ctypes.c_int64()
    if lib().or_width(_ptr(lat, _u8p), Lx, Ly, H0, ctypes.byref(s1), ctypes.byref(s2)) != 0:
        raise OverflowError("width sums exceed int64")
    return s1.value, s2.value


def width_rows(rows: np.ndarray, h_start: int) -> tuple:
    """(S1, S2, h_next) of a band of rows of a larger lattice whose first site
    has height ``h_start``; exact Python integers (no int64 limit).  Summing
    the bands of a lattice in order, each started at the previous band's
    ``h_next`` (the first at H0), gives ``width_sums`` of the whole lattice."""
    _check_lattice(rows)
    n, Lx = rows.shape
    s1l, s2l = ctypes.c_uint64(), ctypes.c_uint64()
    s1h, s2h, hn = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lib().or_width_rows(_ptr(rows, _u8p), Lx, n, int(h_start), ctypes.byref(s1l),
                        ctypes.byref(s1h), ctypes.byref(s2l), ctypes.byref(s2h), ctypes.byref(hn))
    return (s1h.value << 64) + s1l.value, (s2h.value << 64) + s2l.value, hn.value


def w2(S1: int, S2: int, N: int) -> float:
    """W^2 = S2/N - (S1/N)^2 from exact sums (numerator in Python integers)."""
    return (N * S2 - S1 * S1) / (N * N)


def ensemble(Lx: int, Ly: int, p: float, q: float, seed0: int, R: int, tmax: int,
             rsu: bool = False, delayed: bool = False) -> np.ndarray:
    """(S1, S2) after every MCS t = 1..tmax of R flat-start realizations with
    seeds seed0 .. seed0+R-1; returns an int64 array of shape (R, tmax, 2).
    ``rsu`` selects the random-sequential reference, ``delayed`` the tiled
    dynamics with delayed cell borders."""
    return ensemble_at(Lx, Ly, p, q, seed0, R, list(range(1, tmax + 1)), rsu, delayed)


def ensemble_at(Lx: int, Ly: int, p: float, q: float, seed0: int, R: int, times,
                rsu: bool = False, delayed: bool = False) -> np.ndarray:
    """(S1, S2) after MCS ``times`` (increasing, >= 1) of R flat-start
    realizations with seeds seed0 .. seed0+R-1, realizations spread over the
    host threads; an int64 array of shape (R, len(times), 2)."""
    tv = np.ascontiguousarray(np.asarray(times, dtype=np.int64))
    out = np.zeros((R, len(tv), 2), dtype=np.int64)
    kind = 1 if rsu else (2 if delayed else 0)
    rc = lib().or_ensemble_at(Lx, Ly, float(p), float(q), seed0, R, _ptr(tv, _i64p), len(tv),
                              kind, _ptr(out, _i64p))
    if rc != 0:
        raise RuntimeError(f"or_ensemble_at failed ({rc})")
    return out


class Window:
    """The exact state of a rectangle of a large periodic lattice under the
    tiled dynamics (blocks of a sweep are independent, Sec. II).

    ``lat`` holds lattice sites ((wx0 + u) mod Lx, (wy0 + v) mod Ly) at
    ``lat[v, u]``; ``valid`` = (vx0, vy0, vx1, vy1) is the half-open rectangle
    of window coordinates whose state is exact; ``H0`` is the height of site
    (0,0) while it stays inside.  Each ``sweep`` updates the blocks lying
    wholly inside ``valid`` and shrinks it to their union."""

    def __init__(self, lat: np.ndarray, wx0: int, wy0: int, Lx: int, Ly: int, H0: int = 0):
        _check_lattice(lat)
        self.lat, self.wx0, self.wy0, self.Lx, self.Ly, self.H0 = lat, wx0, wy0, Lx, Ly, H0
        self.valid = (0, 0, lat.shape[1], lat.shape[0])

    def sweep(self, p: float, q: float, seed: int, s: int, delayed: bool = False) -> None:
        Wy, Wx = self.lat.shape
        v = [ctypes.c_int64(x) for x in self.valid]
        h = ctypes.c_int64(self.H0)
        rc = lib().or_window_sweep(_ptr(self.lat, _u8p), Wx, Wy, self.wx0, self.wy0, self.Lx,
                                   self.Ly, threshold(p), threshold(q), seed, s,
                                   ctypes.byref(v[0]), ctypes.byref(v[1]), ctypes.byref(v[2]),
                                   ctypes.byref(v[3]), ctypes.byref(h), int(delayed))
        if rc != 0:
            raise ValueError(f"or_window_sweep failed ({rc})")
        self.valid = tuple(x.value for x in v)
        self.H0 = h.value


def flat_window(wx0: int, wy0: int, Wx: int, Wy: int) -> np.ndarray:
    """Sites ((wx0 + u), (wy0 + v)) of the flat zig-zag state (Sec. III) of
    any even-sided periodic lattice: bx = by = [x + y even]."""
    x = (wx0 + np.arange(Wx)) % 2
    y = (wy0 + np.arange(Wy)) % 2
    up = ((x[None, :] + y[:, None]) % 2 == 0).astype(np.uint8)
    return np.ascontiguousarray(up | (up << 1))


def sampling_times(t_max: int, m: float) -> list:
    """Measurement times of Sec. III: t_{i+1} = (t_i + 10) e^m from t_0 = 0,
    each rounded up to a whole MCS, repeats dropped, and t_max itself last."""
    import math

    out, t = [], 0.0
    while True:
        t = (t + 10.0) * math.exp(m)
        if t > t_max:
            break
        c = math.ceil(t)
        if c not in out:
            out.append(c)
    if t_max > 0 and t_max not in out:
        out.append(t_max)
    return out


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))
