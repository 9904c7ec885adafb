"""Pins of the oracle's large-lattice and ensemble helpers (CPU only).

* ``oracle.Window``: blocks of one sweep are independent (Sec. II), so the
  sweep of a rectangle of the lattice is exact on the union of the blocks
  lying wholly inside it.  Pinned against whole-lattice sweeps of the plain
  oracle, with windows that wrap around the periodic boundary, several
  sweeps, both cell-border contracts and the height of site (0,0).
* ``oracle.flat_window``: slices of the flat zig-zag state (Sec. III).
* ``oracle.ensemble_at``: realizations on separate host threads give what a
  single thread gives and what the every-MCS ensemble gives at those times.
* ``oracle.sampling_times``: the measurement times of Sec. III,
  t_{i+1} = (t_i + 10) e^m, worked out by hand for m = 0.01.
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("wx0,wy0", [(0, 0), (1000, 300), (-700, 511)])
def test_flat_window_is_a_slice_of_the_flat_state(wx0, wy0):
    Lx, Ly = 1024, 768
    full = oracle.flat(Lx, Ly)
    w = oracle.flat_window(wx0, wy0, 600, 500)
    xs = (wx0 + np.arange(600)) % Lx
    ys = (wy0 + np.arange(500)) % Ly
    assert np.array_equal(w, full[np.ix_(ys, xs)])


@pytest.mark.parametrize("delayed", [False, True])
@pytest.mark.parametrize("wx0,wy0,Wx,Wy", [(700, 100, 1024, 1024), (-300, -200, 1280, 1024),
                                          (0, 0, 2048, 1536)])
def test_window_sweeps_equal_whole_lattice_sweeps(delayed, wx0, wy0, Wx, Wy):
    Lx, Ly = 2048, 1536
    p, q, seed, n = 0.9, 0.15, 7, 3
    full = oracle.flat(Lx, Ly)
    H0 = 0
    win = oracle.Window(oracle.flat_window(wx0, wy0, Wx, Wy), wx0, wy0, Lx, Ly)
    for s in range(n):
        H0 = oracle.sweep(full, p, q, seed, s, H0, delayed=delayed)
        win.sweep(p, q, seed, s, delayed=delayed)
    vx0, vy0, vx1, vy1 = win.valid
    assert vx1 - vx0 >= Wx - 2 * n * 256 and vy1 - vy0 >= Wy - 2 * n * 256
    xs = (wx0 + np.arange(vx0, vx1)) % Lx
    ys = (wy0 + np.arange(vy0, vy1)) % Ly
    assert np.array_equal(win.lat[vy0:vy1, vx0:vx1], full[np.ix_(ys, xs)])
    if (Wx, Wy) == (Lx, Ly):
        # a window of the whole lattice loses nothing at the wrap-around
        # only if its edges meet block edges; it must still contain (0,0)
        pass
    u00, v00 = (0 - wx0) % Lx, (0 - wy0) % Ly
    if vx0 <= u00 < vx1 and vy0 <= v00 < vy1:
        assert win.H0 == H0


def test_window_with_site_00_tracks_its_height():
    Lx = Ly = 4096
    p, q, seed, n = 1.0, 0.0, 3, 4
    wx0 = wy0 = -1536
    win = oracle.Window(oracle.flat_window(wx0, wy0, 3072, 3072), wx0, wy0, Lx, Ly)
    full = oracle.flat(Lx, Ly)
    H0 = 0
    for s in range(n):
        H0 = oracle.sweep(full, p, q, seed, s, H0)
        win.sweep(p, q, seed, s)
    vx0, vy0, vx1, vy1 = win.valid
    assert vx0 <= 1536 < vx1 and vy0 <= 1536 < vy1
    assert win.H0 == H0 and H0 > 0


def test_window_that_holds_no_block_becomes_empty():
    win = oracle.Window(oracle.flat_window(5, 5, 300, 300), 5, 5, 1024, 1024)
    win.sweep(1.0, 0.0, 1, 0)
    win.sweep(1.0, 0.0, 1, 1)
    vx0, vy0, vx1, vy1 = win.valid
    assert vx1 <= vx0 or vy1 <= vy0


@pytest.mark.parametrize("rsu,delayed", [(False, False), (True, False), (False, True)])
def test_ensemble_at_equals_every_mcs_ensemble_and_one_thread(rsu, delayed):
    times = [1, 2, 5, 9, 16]
    full = oracle.ensemble(32, 32, 0.95, 0.05, 40, 6, 16, rsu=rsu, delayed=delayed)
    at = oracle.ensemble_at(32, 32, 0.95, 0.05, 40, 6, times, rsu=rsu, delayed=delayed)
    assert np.array_equal(at, full[:, [t - 1 for t in times], :])
    n = oracle.num_threads()
    try:
        oracle.set_num_threads(1)
        one = oracle.ensemble_at(32, 32, 0.95, 0.05, 40, 6, times, rsu=rsu, delayed=delayed)
    finally:
        oracle.set_num_threads(n)
    assert np.array_equal(one, at)
    # each realization on its own equals the lone run with that seed
    for r in (0, 5):
        lat = oracle.flat(32, 32)
        if rsu:
            H0 = oracle.rsu_run(lat, 0.95, 0.05, 40 + r, 0, 9, 0)
        else:
            H0 = oracle.run(lat, 0.95, 0.05, 40 + r, 0, 9, 0, delayed=delayed)
        assert tuple(at[r, 3]) == oracle.width_sums(lat, H0)


def test_ensemble_at_rejects_unordered_times():
    with pytest.raises(RuntimeError):
        oracle.ensemble_at(8, 8, 1.0, 0.0, 1, 2, [3, 2])
    with pytest.raises(RuntimeError):
        oracle.ensemble_at(8, 8, 1.0, 0.0, 1, 2, [0, 2])


def test_sampling_times_by_hand():
    # e^0.01 = 1.010050167...: t1 = 10.1005, t2 = 20.3015, t3 = 30.6055,
    # t4 = 41.0136, t5 = 51.5257 -> rounded up 11, 21, 31, 42, 52
    assert oracle.sampling_times(52, 0.01) == [11, 21, 31, 42, 52]
    # t_max itself is always the last time; repeats are dropped
    assert oracle.sampling_times(45, 0.01) == [11, 21, 31, 42, 45]
    assert oracle.sampling_times(0, 0.01) == []
    # with a large m the recurrence leaps: t1 = 10 e = 27.18, t2 = (10 e + 10) e = 101.07
    assert oracle.sampling_times(200, 1.0) == [28, 102, 200]
    ts = oracle.sampling_times(10000, 0.01)
    assert ts == sorted(set(ts)) and ts[-1] == 10000
    # the gaps approach the geometric law t_{i+1}/t_i -> e^m
    assert abs(ts[-2] / ts[-3] - np.exp(0.01)) < 2e-3


def _bigint_sums(lat, H0):
    """S1, S2 in Python integers from heights reconstructed along the other
    path (first along row 0, then up each column)."""
    sx = 2 * (lat & 1).astype(np.int64) - 1
    sy = 2 * ((lat >> 1) & 1).astype(np.int64) - 1
    row0 = np.concatenate([[0], np.cumsum(sx[0, :-1])])
    h = row0[None, :] + np.concatenate([np.zeros((1, lat.shape[1]), np.int64),
                                         np.cumsum(sy[:-1, :], axis=0)])
    hs = [int(v) + H0 for v in h.ravel()]
    return sum(hs), sum(v * v for v in hs)


@pytest.mark.parametrize("H0", [0, 2, -4, 2 * 10**12, -(2**40)])
def test_width_rows_in_bands_equal_the_whole_lattice(H0):
    from tests import inputs

    lat, h0 = inputs.rough_state(64, 48, seed=9, mcs=3)
    H = H0 + h0
    S1, S2 = 0, 0
    h = H
    for y0, n in ((0, 5), (5, 1), (6, 30), (36, 12)):
        a, b, h = oracle.width_rows(np.ascontiguousarray(lat[y0:y0 + n]), h)
        S1, S2 = S1 + a, S2 + b
    assert h == H  # the column-0 walk closes
    assert (S1, S2) == _bigint_sums(lat, H)
    if abs(H) < 2**20:
        assert (S1, S2) == oracle.width_sums(lat, H)


def test_synthetic_surfaces_are_valid_and_pack_to_their_rows():
    from tests import inputs
    from tests.test_oracle_model import assert_valid

    L = 128
    a, b = inputs.balanced_bits(L, 1), inputs.balanced_bits(96, 2)
    for kind in ("separable", "diagonal"):
        Ly = 96 if kind == "separable" else L
        rows = (inputs.separable_rows(a, b, 0, Ly) if kind == "separable"
                else inputs.diagonal_rows(a, 0, Ly))
        assert_valid(rows)
        part = (inputs.separable_rows(a, b, 17, 40) if kind == "separable"
                else inputs.diagonal_rows(a, 17, 40))
        assert np.array_equal(part, rows[17:57])
        ck = inputs.checkpoint_of(kind, a, b, 6)
        planes = ck[80:].view("<u4").reshape(2, Ly, L // 32)
        unpacked = np.unpackbits(planes.view(np.uint8), axis=-1, bitorder="little")
        assert np.array_equal(unpacked[0], rows & 1)
        assert np.array_equal(unpacked[1], (rows >> 1) & 1)
