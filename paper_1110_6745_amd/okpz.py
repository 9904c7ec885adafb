"""Python binding of the okpz C ABI (``include/okpz.h``).

Argument marshalling only: every step of the hot path runs in the HIP
library ``libokpz.so`` built in this directory.  Importing this module fails
loudly if the library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch is the memory/stream layer of this package.  Importing it first makes
# the process load one HIP runtime (torch's); the library then binds to it by
# its soname instead of loading a second runtime.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libokpz.so")

OKPZ_OK = 0
OKPZ_EINVAL = -22
OKPZ_ENOMEM = -12
OKPZ_EOVERFLOW = -75
OKPZ_EDEVICE = -5
OKPZ_EBUSY = -16
OKPZ_CELLS_DEAD = 0
OKPZ_CELLS_DELAYED = 1


class OkpzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"okpz error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"okpz HIP library not built: {LIB_PATH} is missing "
                      "(run __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_sz = ctypes.c_size_t


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("okpz_geometry", ctypes.c_int, _i64, _i64, _i32p, _i32p, _i32p)
_sig("okpz_required_bytes", _sz, _i64, _i64)
_sig("okpz_init", ctypes.c_int, ctypes.POINTER(_vp), _i64, _i64, ctypes.c_double,
     ctypes.c_double, ctypes.c_uint64)
_sig("okpz_init_on", ctypes.c_int, ctypes.POINTER(_vp), _i64, _i64, ctypes.c_double,
     ctypes.c_double, ctypes.c_uint64, _vp, _sz, _vp)
_sig("okpz_required_bytes_in_place", _sz, _i64, _i64)
_sig("okpz_init_in_place", ctypes.c_int, ctypes.POINTER(_vp), _i64, _i64, ctypes.c_double,
     ctypes.c_double, ctypes.c_uint64, _vp, _sz, _vp)
_sig("okpz_get_copies", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_int32))
_sig("okpz_sweep", ctypes.c_int, _vp, _i64)
_sig("okpz_width", ctypes.c_int, _vp, _i64, _i64p, _i64p)
_sig("okpz_w2", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double))
_sig("okpz_psd", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))
_sig("okpz_psd_noalloc", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double),
     ctypes.POINTER(ctypes.c_double))
_sig("okpz_time", ctypes.c_int, _vp, _i64p)
_sig("okpz_h0", ctypes.c_int, _vp, _i64p)
_sig("okpz_stream", _vp, _vp)
_sig("okpz_get_lattice", ctypes.c_int, _vp, _u8p, _sz)
_sig("okpz_get_rows", ctypes.c_int, _vp, _i64, _i64, _u8p, _sz)
_sig("okpz_set_lattice", ctypes.c_int, _vp, _u8p, _sz, _i64, _i64)
_sig("okpz_save", ctypes.c_int, _vp, _vp, ctypes.POINTER(_sz))
_sig("okpz_load", ctypes.c_int, ctypes.POINTER(_vp), _vp, _sz)
_sig("okpz_set_threads", ctypes.c_int, _vp, ctypes.c_int)
_sig("okpz_set_cell_borders", ctypes.c_int, _vp, ctypes.c_int32)
_sig("okpz_batch_set_cell_borders", ctypes.c_int, _vp, ctypes.c_int32)
_sig("okpz_batch_get_cell_borders", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_int32))
_sig("okpz_get_cell_borders", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_int32))
_sig("okpz_sync", ctypes.c_int, _vp)
_sig("okpz_free", ctypes.c_int, _vp)
_sig("okpz_last_error", ctypes.c_char_p)
_sig("okpz_sampling_times", ctypes.c_int, _i64, ctypes.c_double, _i64p, _i64, _i64p)

class OkpzJob(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int64), ("Ly", ctypes.c_int64), ("p", ctypes.c_double),
                ("q", ctypes.c_double), ("seed", ctypes.c_uint64), ("t_max", ctypes.c_int64)]


_jobp = ctypes.POINTER(OkpzJob)
_sig("okpz_batch_create", ctypes.c_int, ctypes.POINTER(_vp), _jobp, ctypes.c_int32,
     ctypes.c_double)
_sig("okpz_batch_set_mapping", ctypes.c_int, _vp, ctypes.c_int32, ctypes.c_int32)
_sig("okpz_batch_get_mapping", ctypes.c_int, _vp, _i32p, _i32p)
_sig("okpz_batch_autotune", ctypes.c_int, _vp, _i64, _i32p, _i32p)
_sig("okpz_batch_run", ctypes.c_int, _vp)
_sig("okpz_batch_start", ctypes.c_int, _vp)
_sig("okpz_batch_run_for", ctypes.c_int, _vp, ctypes.c_double, _i32p)
_sig("okpz_batch_last_ms", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_float))
_sig("okpz_batch_samples", ctypes.c_int, _vp, ctypes.c_int32, _i64p, _i64p, _i64p,
     ctypes.c_int32, _i32p)
_sig("okpz_batch_get_lattice", ctypes.c_int, _vp, ctypes.c_int32, _u8p, _sz)
_sig("okpz_batch_h0", ctypes.c_int, _vp, ctypes.c_int32, _i64p)
_sig("okpz_batch_w2_histogram", ctypes.c_int, _vp, _i64, _i64, _i64, ctypes.c_double,
     ctypes.c_double, ctypes.c_int32, _i64p, _i64p, _i64p)
_dp = ctypes.POINTER(ctypes.c_double)
_sig("okpz_batch_w2_cumulants", ctypes.c_int, _vp, _i64, _i64, _i64, _i64p, _dp, _dp)
_sig("okpz_batch_psi", ctypes.c_int, _vp, _i64, _i64, _i64, ctypes.c_double, ctypes.c_int32, _dp,
     _i64p)
_sig("okpz_batch_free", ctypes.c_int, _vp)
_sig("okpz_batch_last_error", ctypes.c_char_p)

_sig("okpz_serve_create", ctypes.c_int, ctypes.POINTER(_vp), _sz, ctypes.c_int32, _i64,
     ctypes.c_double)
_sig("okpz_serve_set_mapping", ctypes.c_int, _vp, ctypes.c_int32, ctypes.c_int32)
_sig("okpz_serve_set_cell_borders", ctypes.c_int, _vp, ctypes.c_int32)
_sig("okpz_serve_get_cell_borders", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_int32))
_sig("okpz_serve_now", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double))
_sig("okpz_serve_submit", ctypes.c_int, _vp, _jobp, ctypes.c_double, ctypes.c_int32, _i64p)
_sig("okpz_serve_step", ctypes.c_int, _vp, _i32p, _i32p)
_sig("okpz_serve_job", ctypes.c_int, _vp, _i64, _i32p, ctypes.POINTER(ctypes.c_double),
     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))
_sig("okpz_serve_cancel", ctypes.c_int, _vp, _i64)
_sig("okpz_serve_samples", ctypes.c_int, _vp, _i64, _i64p, _i64p, _i64p, ctypes.c_int32, _i32p)
_sig("okpz_serve_result", ctypes.c_int, _vp, _i64, _u8p, _sz, _i64p)
_sig("okpz_serve_stats", ctypes.c_int, _vp, _i64p, ctypes.POINTER(ctypes.c_double), _i64p,
     ctypes.POINTER(_sz))
_sig("okpz_serve_free", ctypes.c_int, _vp)

EXPORTED = ["okpz_geometry", "okpz_required_bytes", "okpz_init", "okpz_init_on",
            "okpz_required_bytes_in_place", "okpz_init_in_place", "okpz_get_copies", "okpz_sweep",
            "okpz_width", "okpz_w2", "okpz_psd", "okpz_psd_noalloc", "okpz_time", "okpz_h0", "okpz_stream", "okpz_get_lattice",
            "okpz_get_rows", "okpz_set_lattice", "okpz_save", "okpz_load", "okpz_set_threads",
            "okpz_set_cell_borders", "okpz_get_cell_borders", "okpz_sync",
            "okpz_free", "okpz_last_error", "okpz_sampling_times", "okpz_batch_create",
            "okpz_batch_set_mapping",
            "okpz_batch_get_mapping", "okpz_batch_set_cell_borders",
            "okpz_batch_get_cell_borders", "okpz_batch_autotune", "okpz_batch_run", "okpz_batch_start", "okpz_batch_run_for",
            "okpz_batch_last_ms", "okpz_batch_samples", "okpz_batch_get_lattice", "okpz_batch_h0",
            "okpz_batch_w2_histogram", "okpz_batch_w2_cumulants", "okpz_batch_psi",
            "okpz_serve_create", "okpz_serve_set_mapping", "okpz_serve_set_cell_borders",
            "okpz_serve_get_cell_borders",
            "okpz_serve_now", "okpz_serve_submit", "okpz_serve_step", "okpz_serve_job",
            "okpz_serve_cancel", "okpz_serve_samples", "okpz_serve_result", "okpz_serve_stats", "okpz_serve_free",
            "okpz_batch_free", "okpz_batch_last_error"]


def _check(rc: int) -> None:
    if rc != OKPZ_OK:
        raise OkpzError(rc, _lib.okpz_last_error().decode(errors="replace"))


def lib() -> ctypes.CDLL:
    return _lib


# ---- functions with the C names -------------------------------------------
def okpz_geometry(Lx: int, Ly: int) -> tuple:
    bx, by, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.okpz_geometry(Lx, Ly, ctypes.byref(bx), ctypes.byref(by), ctypes.byref(c)))
    return bx.value, by.value, c.value


def okpz_required_bytes(Lx: int, Ly: int) -> int:
    return int(_lib.okpz_required_bytes(Lx, Ly))


def okpz_init(Lx: int, Ly: int, p: float, q: float, seed: int) -> "Sim":
    h = _vp()
    _check(_lib.okpz_init(ctypes.byref(h), Lx, Ly, float(p), float(q), int(seed)))
    return Sim(h, Lx, Ly)


def okpz_init_on(Lx: int, Ly: int, p: float, q: float, seed: int, dev_ptr: int, nbytes: int,
                 stream_ptr: int | None) -> "Sim":
    h = _vp()
    _check(_lib.okpz_init_on(ctypes.byref(h), Lx, Ly, float(p), float(q), int(seed),
                             _vp(dev_ptr), nbytes, _vp(stream_ptr or 0)))
    return Sim(h, Lx, Ly)


def okpz_required_bytes_in_place(Lx: int, Ly: int) -> int:
    return int(_lib.okpz_required_bytes_in_place(Lx, Ly))


def okpz_init_in_place(Lx: int, Ly: int, p: float, q: float, seed: int, dev_ptr: int = 0,
                       nbytes: int = 0, stream_ptr: int | None = None) -> "Sim":
    """One lattice copy updated in place (dev_ptr 0: the library allocates)."""
    h = _vp()
    _check(_lib.okpz_init_in_place(ctypes.byref(h), Lx, Ly, float(p), float(q), int(seed),
                                   _vp(dev_ptr or 0), nbytes, _vp(stream_ptr or 0)))
    return Sim(h, Lx, Ly)


def okpz_load(buf) -> "Sim":
    """A checkpoint from any bytes-like object (bytes, bytearray, uint8 array),
    passed without a copy."""
    h = _vp()
    view = np.frombuffer(buf, dtype=np.uint8)
    _check(_lib.okpz_load(ctypes.byref(h), _vp(view.ctypes.data), view.nbytes))
    sim = Sim(h, 0, 0)
    sim.Ly, sim.Lx = sim._shape_from_lattice_size(buf)
    return sim


class Sim:
    """One simulated lattice (a handle of the C library)."""

    def __init__(self, handle, Lx: int, Ly: int):
        self._h = handle
        self.Lx, self.Ly = Lx, Ly
        self._keep = None  # caller-owned buffer kept alive with the handle

    @staticmethod
    def _shape_from_lattice_size(buf: bytes) -> tuple:
        Lx, Ly = np.frombuffer(buf[16:32], dtype=np.int64)
        return int(Ly), int(Lx)

    @property
    def handle(self):
        return self._h

    def sweep(self, n_mcs: int) -> None:
        _check(_lib.okpz_sweep(self._h, int(n_mcs)))

    def width(self, t: int | None = None) -> tuple:
        """(sum_h, sum_h2) at MCS t (default: now), exact integers."""
        if t is None:
            t = self.time()
        s1, s2 = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.okpz_width(self._h, int(t), ctypes.byref(s1), ctypes.byref(s2)))
        return s1.value, s2.value

    def w2(self) -> float:
        v = ctypes.c_double()
        _check(_lib.okpz_w2(self._h, ctypes.byref(v)))
        return v.value

    def psd(self) -> tuple:
        """(Sx, Sy): the surface's power spectrum along the x axis for
        k = 2 pi n / Lx, n = 0 .. Lx/2, and along the y axis for n = 0 .. Ly/2
        (Eqs. (PSD), (hF))."""
        Lx, Ly = self.Lx, self.Ly
        sx = np.empty(Lx // 2 + 1, dtype=np.float64)
        sy = np.empty(Ly // 2 + 1, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(_lib.okpz_psd(self._h, sx.ctypes.data_as(dp), sy.ctypes.data_as(dp)))
        return sx, sy

    def psd_noalloc(self) -> tuple:
        """As psd(), through okpz_psd_noalloc: no device allocation, the
        library's fixed per-GPU scratch (sides up to 2^17)."""
        Lx, Ly = self.Lx, self.Ly
        sx = np.empty(Lx // 2 + 1, dtype=np.float64)
        sy = np.empty(Ly // 2 + 1, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(_lib.okpz_psd_noalloc(self._h, sx.ctypes.data_as(dp), sy.ctypes.data_as(dp)))
        return sx, sy

    def time(self) -> int:
        t = ctypes.c_int64()
        _check(_lib.okpz_time(self._h, ctypes.byref(t)))
        return t.value

    def h0(self) -> int:
        v = ctypes.c_int64()
        _check(_lib.okpz_h0(self._h, ctypes.byref(v)))
        return v.value

    def stream(self) -> int:
        return _lib.okpz_stream(self._h) or 0

    def get_lattice(self) -> np.ndarray:
        out = np.empty((self.Ly, self.Lx), dtype=np.uint8)
        _check(_lib.okpz_get_lattice(self._h, out.ctypes.data_as(_u8p), out.nbytes))
        return out

    def get_rows(self, y0: int, nrows: int) -> np.ndarray:
        out = np.empty((nrows, self.Lx), dtype=np.uint8)
        _check(_lib.okpz_get_rows(self._h, int(y0), int(nrows), out.ctypes.data_as(_u8p),
                                  out.nbytes))
        return out

    def set_lattice(self, lat: np.ndarray, H0: int, t: int) -> None:
        lat = np.ascontiguousarray(lat, dtype=np.uint8)
        if lat.shape != (self.Ly, self.Lx):
            raise ValueError(f"lattice shape {lat.shape} != {(self.Ly, self.Lx)}")
        _check(_lib.okpz_set_lattice(self._h, lat.ctypes.data_as(_u8p), lat.nbytes, int(H0),
                                     int(t)))

    def save(self) -> bytes:
        n = _sz(0)
        _check(_lib.okpz_save(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(_lib.okpz_save(self._h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def set_threads(self, threads: int) -> None:
        _check(_lib.okpz_set_threads(self._h, int(threads)))

    def set_cell_borders(self, kind: int) -> None:
        """OKPZ_CELLS_DEAD (default) or OKPZ_CELLS_DELAYED (Sec. II)."""
        _check(_lib.okpz_set_cell_borders(self._h, int(kind)))

    def cell_borders(self) -> int:
        k = ctypes.c_int32()
        _check(_lib.okpz_get_cell_borders(self._h, ctypes.byref(k)))
        return k.value

    def copies(self) -> int:
        c = ctypes.c_int32()
        _check(_lib.okpz_get_copies(self._h, ctypes.byref(c)))
        return c.value

    def sync(self) -> None:
        _check(_lib.okpz_sync(self._h))

    def free(self) -> None:
        if self._h:
            _check(_lib.okpz_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _bcheck(rc: int) -> None:
    if rc != OKPZ_OK:
        raise OkpzError(rc, _lib.okpz_batch_last_error().decode(errors="replace"))


class Batch:
    """Many independent realizations run in one persistent launch.

    ``jobs``: iterable of (Lx, Ly, p, q, seed, t_max); ``m``: exponent of the
    sampling times t_{i+1} = (t_i + 10) e^m.
    """

    def __init__(self, jobs, m: float = 0.01):
        arr = (OkpzJob * len(jobs))()
        for i, (Lx, Ly, p, q, seed, t_max) in enumerate(jobs):
            arr[i] = OkpzJob(int(Lx), int(Ly), float(p), float(q), int(seed), int(t_max))
        self.jobs = [tuple(j) for j in jobs]
        h = _vp()
        _bcheck(_lib.okpz_batch_create(ctypes.byref(h), arr, len(jobs), float(m)))
        self._h = h

    def set_mapping(self, threads: int, workgroups: int = 0) -> None:
        _bcheck(_lib.okpz_batch_set_mapping(self._h, int(threads), int(workgroups)))

    def set_cell_borders(self, kind: int) -> None:
        """OKPZ_CELLS_DEAD (default) or OKPZ_CELLS_DELAYED for every job."""
        _bcheck(_lib.okpz_batch_set_cell_borders(self._h, int(kind)))

    def cell_borders(self) -> int:
        k = ctypes.c_int32()
        _bcheck(_lib.okpz_batch_get_cell_borders(self._h, ctypes.byref(k)))
        return k.value

    def mapping(self) -> tuple:
        t, w = ctypes.c_int32(), ctypes.c_int32()
        _bcheck(_lib.okpz_batch_get_mapping(self._h, ctypes.byref(t), ctypes.byref(w)))
        return t.value, w.value

    def autotune(self, trial_mcs: int) -> tuple:
        """Time each (threads, workgroups) candidate on the workload scaled so
        that the longest job runs trial_mcs sweeps; keep and return the best."""
        t, w = ctypes.c_int32(), ctypes.c_int32()
        _bcheck(_lib.okpz_batch_autotune(self._h, int(trial_mcs), ctypes.byref(t),
                                         ctypes.byref(w)))
        return t.value, w.value

    def run(self, slice_ms: float | None = None, progress=None) -> float:
        """Run all jobs to t_max; returns the device time in ms.  With
        slice_ms, the run goes in slices of about that many milliseconds
        (okpz_batch_start / okpz_batch_run_for), calling progress(finished)
        after each slice."""
        if slice_ms is None:
            _bcheck(_lib.okpz_batch_run(self._h))
        else:
            _bcheck(_lib.okpz_batch_start(self._h))
            done = ctypes.c_int32(0)
            while True:
                _bcheck(_lib.okpz_batch_run_for(self._h, float(slice_ms), ctypes.byref(done)))
                if progress is not None:
                    progress(done.value)
                if done.value == len(self.jobs):
                    break
        ms = ctypes.c_float()
        _bcheck(_lib.okpz_batch_last_ms(self._h, ctypes.byref(ms)))
        return ms.value

    def samples(self, job: int):
        n = ctypes.c_int32()
        _bcheck(_lib.okpz_batch_samples(self._h, job, None, None, None, 0, ctypes.byref(n)))
        t = np.zeros(n.value, dtype=np.int64)
        s1 = np.zeros(n.value, dtype=np.int64)
        s2 = np.zeros(n.value, dtype=np.int64)
        _bcheck(_lib.okpz_batch_samples(self._h, job, t.ctypes.data_as(_i64p),
                                        s1.ctypes.data_as(_i64p), s2.ctypes.data_as(_i64p),
                                        n.value, ctypes.byref(n)))
        return t, s1, s2

    def get_lattice(self, job: int) -> np.ndarray:
        Lx, Ly = self.jobs[job][0], self.jobs[job][1]
        out = np.empty((Ly, Lx), dtype=np.uint8)
        _bcheck(_lib.okpz_batch_get_lattice(self._h, job, out.ctypes.data_as(_u8p), out.nbytes))
        return out

    def h0(self, job: int) -> int:
        v = ctypes.c_int64()
        _bcheck(_lib.okpz_batch_h0(self._h, job, ctypes.byref(v)))
        return v.value

    def w2_histogram(self, Lx: int, Ly: int, t_from: int, lo: float, hi: float, nbins: int):
        """(counts, under, over) of the W^2 samples with t >= t_from of size Lx x Ly."""
        counts = np.zeros(nbins, dtype=np.int64)
        u, o = ctypes.c_int64(), ctypes.c_int64()
        _bcheck(_lib.okpz_batch_w2_histogram(self._h, Lx, Ly, t_from, float(lo), float(hi), nbins,
                                             counts.ctypes.data_as(_i64p), ctypes.byref(u),
                                             ctypes.byref(o)))
        return counts, u.value, o.value

    def w2_cumulants(self, Lx: int, Ly: int, t_from: int):
        """(count, nu[4], kappa[4]): moments and cumulants of W^2 over the
        samples with t >= t_from of size Lx x Ly (okpz_batch_w2_cumulants)."""
        n = ctypes.c_int64()
        nu = np.zeros(4)
        kappa = np.zeros(4)
        _bcheck(_lib.okpz_batch_w2_cumulants(self._h, Lx, Ly, t_from, ctypes.byref(n),
                                             nu.ctypes.data_as(_dp), kappa.ctypes.data_as(_dp)))
        return n.value, nu, kappa

    def psi(self, Lx: int, Ly: int, t_from: int, x_hi: float, nbins: int):
        """(psi[nbins], count): density of W^2 / <W^2> on [0, x_hi) (okpz_batch_psi)."""
        out = np.zeros(nbins)
        n = ctypes.c_int64()
        _bcheck(_lib.okpz_batch_psi(self._h, Lx, Ly, t_from, float(x_hi), nbins,
                                    out.ctypes.data_as(_dp), ctypes.byref(n)))
        return out, n.value

    def free(self) -> None:
        if self._h:
            _bcheck(_lib.okpz_batch_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sampling_times(t_max: int, m: float) -> list:
    """Measurement times of Sec. III (okpz_sampling_times)."""
    n = ctypes.c_int64()
    _check(_lib.okpz_sampling_times(int(t_max), float(m), None, 0, ctypes.byref(n)))
    out = (ctypes.c_int64 * max(n.value, 1))()
    _check(_lib.okpz_sampling_times(int(t_max), float(m), out, n.value, ctypes.byref(n)))
    return [int(v) for v in out[:n.value]]


class Server:
    """Continuous batching of simulation jobs (see okpz_serve_* in okpz.h)."""

    def __init__(self, hbm_budget: int, max_slots: int = 64, quantum_sites: int = 1 << 31,
                 m: float = 0.01):
        h = _vp()
        _bcheck(_lib.okpz_serve_create(ctypes.byref(h), int(hbm_budget), int(max_slots),
                                       int(quantum_sites), float(m)))
        self._h = h
        self.jobs = {}

    def set_mapping(self, threads: int, workgroups: int = 0) -> None:
        _bcheck(_lib.okpz_serve_set_mapping(self._h, int(threads), int(workgroups)))

    def set_cell_borders(self, kind: int) -> None:
        """OKPZ_CELLS_DEAD (default) or OKPZ_CELLS_DELAYED, before the first submit."""
        _bcheck(_lib.okpz_serve_set_cell_borders(self._h, int(kind)))

    def cell_borders(self) -> int:
        k = ctypes.c_int32()
        _bcheck(_lib.okpz_serve_get_cell_borders(self._h, ctypes.byref(k)))
        return k.value

    def now(self) -> float:
        v = ctypes.c_double()
        _bcheck(_lib.okpz_serve_now(self._h, ctypes.byref(v)))
        return v.value

    def submit(self, job, arrival: float = -1.0, keep_lattice: bool = False) -> int:
        Lx, Ly, p, q, seed, t_max = job
        j = OkpzJob(int(Lx), int(Ly), float(p), float(q), int(seed), int(t_max))
        i = ctypes.c_int64()
        _bcheck(_lib.okpz_serve_submit(self._h, ctypes.byref(j), float(arrival), int(keep_lattice),
                                       ctypes.byref(i)))
        self.jobs[i.value] = tuple(job)
        return i.value

    def step(self) -> tuple:
        r, w = ctypes.c_int32(), ctypes.c_int32()
        _bcheck(_lib.okpz_serve_step(self._h, ctypes.byref(r), ctypes.byref(w)))
        return r.value, w.value

    def job(self, i: int) -> dict:
        st = ctypes.c_int32()
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _bcheck(_lib.okpz_serve_job(self._h, i, ctypes.byref(st), ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)))
        return {"state": st.value, "arrival": a.value, "admit": b.value, "finish": c.value}

    def cancel(self, i: int) -> None:
        """Withdraw job i (okpz_serve_cancel): never admitted if waiting,
        retired at once with its samples so far if running."""
        _bcheck(_lib.okpz_serve_cancel(self._h, int(i)))

    def samples(self, i: int):
        n = ctypes.c_int32()
        _bcheck(_lib.okpz_serve_samples(self._h, i, None, None, None, 0, ctypes.byref(n)))
        t = np.zeros(n.value, dtype=np.int64)
        s1 = np.zeros(n.value, dtype=np.int64)
        s2 = np.zeros(n.value, dtype=np.int64)
        _bcheck(_lib.okpz_serve_samples(self._h, i, t.ctypes.data_as(_i64p),
                                        s1.ctypes.data_as(_i64p), s2.ctypes.data_as(_i64p),
                                        n.value, ctypes.byref(n)))
        return t, s1, s2

    def result(self, i: int, lattice: bool = False):
        Lx, Ly = self.jobs[i][0], self.jobs[i][1]
        h0 = ctypes.c_int64()
        if lattice:
            out = np.empty((Ly, Lx), dtype=np.uint8)
            _bcheck(_lib.okpz_serve_result(self._h, i, out.ctypes.data_as(_u8p), out.nbytes,
                                           ctypes.byref(h0)))
            return out, h0.value
        _bcheck(_lib.okpz_serve_result(self._h, i, None, 0, ctypes.byref(h0)))
        return None, h0.value

    def stats(self) -> dict:
        q, d, b = ctypes.c_int64(), ctypes.c_int64(), _sz()
        ms = ctypes.c_double()
        _bcheck(_lib.okpz_serve_stats(self._h, ctypes.byref(q), ctypes.byref(ms), ctypes.byref(d),
                                      ctypes.byref(b)))
        return {"quanta": q.value, "device_ms": ms.value, "done": d.value, "bytes": b.value}

    def drain(self, timeout_s: float = 600.0) -> None:
        """Run quanta until every submitted job is done (sleeping until the
        next arrival when nothing is resident)."""
        import time

        t_end = self.now() + timeout_s
        while True:
            running, waiting = self.step()
            if running == 0 and waiting == 0:
                return
            if running == 0:
                nxt = min(self.job(i)["arrival"] for i in self.jobs if self.job(i)["state"] == 0)
                time.sleep(max(0.0, min(0.05, nxt - self.now())))
            if self.now() > t_end:
                raise TimeoutError("serving did not drain in time")

    def free(self) -> None:
        if self._h:
            _bcheck(_lib.okpz_serve_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def job_stream(n: int, rate: float, seed: int, sizes=(64, 8192), t_range=(1000, 10000)):
    """Synthetic served job stream: Poisson arrivals at `rate` jobs/s; L a
    power of two log-uniform in `sizes`; p uniform in [0.6, 1]; q = 0 or
    1 - p with probability 1/2; t_max log-uniform in `t_range`; job seed =
    index + 1.  Returns [(arrival_s, (L, L, p, q, seed, t_max)), ...]."""
    rng = np.random.default_rng(seed)
    lo, hi = int(np.log2(sizes[0])), int(np.log2(sizes[1]))
    t, out = 0.0, []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        L = 1 << int(rng.integers(lo, hi + 1))
        p = float(rng.uniform(0.6, 1.0))
        q = 0.0 if rng.random() < 0.5 else 1.0 - p
        tm = int(round(np.exp(rng.uniform(np.log(t_range[0]), np.log(t_range[1])))))
        out.append((t, (L, L, p, q, i + 1, tm)))
    return out
