"""Pins of the oracle's dynamics and width against what the paper and the
mathematics of the model fix (CPU only).

* flat zig-zag start: W^2 = 1/4 exactly (Sec. III);
* heights are single valued on the torus: zero row/column slope sums and
  closed plaquettes after every sweep (Sec. I reconstruction, Sec. II
  periodic boundaries);
* each accepted move changes one height by +-2 (Eq. (1)), so
  S1 - S1(0) = 2 (attachments - detachments); with q = 0 the mean height
  never decreases;
* p = q = 0 is the identity; complementing all bits and swapping p and q
  mirrors the trajectory bit for bit (Eq. (1) is symmetric under h -> -h);
* two sites attempted in one step never share a bond (Sec. II dead borders).
"""
import numpy as np
import pytest

import oracle
from tests import inputs


def sx_sy(lat):
    bx = (lat & 1).astype(np.int64)
    by = ((lat >> 1) & 1).astype(np.int64)
    return 2 * bx - 1, 2 * by - 1


def assert_valid(lat):
    sx, sy = sx_sy(lat)
    assert np.all(sx.sum(axis=1) == 0), "row slope sums must vanish"
    assert np.all(sy.sum(axis=0) == 0), "column slope sums must vanish"
    # plaquette (x,y)-(x+1,y)-(x+1,y+1)-(x,y+1) closes
    curl = sx + np.roll(sy, -1, axis=1) - np.roll(sx, -1, axis=0) - sy
    assert np.all(curl == 0), "plaquettes must close"


def heights_numpy(lat, H0):
    """Independent reconstruction along the other path: first along row 0,
    then up each column."""
    sx, sy = sx_sy(lat)
    Ly, Lx = lat.shape
    row0 = H0 + np.concatenate([[0], np.cumsum(sx[0, :-1])])
    h = np.empty((Ly, Lx), dtype=np.int64)
    h[0] = row0
    h[1:] = row0[None, :] + np.cumsum(sy[:-1, :], axis=0)
    return h


@pytest.mark.parametrize("Lx,Ly", [(4, 4), (8, 8), (12, 20), (64, 32), (256, 256)])
def test_flat_state_closed_form(Lx, Ly):
    lat = oracle.flat(Lx, Ly)
    assert_valid(lat)
    N = Lx * Ly
    S1, S2 = oracle.width_sums(lat, 0)
    assert S1 == N // 2 and S2 == N // 2
    # W^2(L,0) = 1/4 exactly: 4 (N S2 - S1^2) = N^2 ; excess width 0
    assert 4 * (N * S2 - S1 * S1) == N * N
    h = oracle.heights(lat, 0)
    xx, yy = np.meshgrid(np.arange(Lx), np.arange(Ly))
    assert np.array_equal(h, (xx + yy) % 2)


def test_width_matches_direct_definition_on_rough_states():
    for (Lx, Ly), seed in [((16, 16), 1), ((32, 12), 2), ((64, 64), 3)]:
        lat, H0 = inputs.rough_state(Lx, Ly, seed, mcs=5)
        assert_valid(lat)
        h = heights_numpy(lat, H0)
        assert np.array_equal(oracle.heights(lat, H0), h)
        S1, S2 = oracle.width_sums(lat, H0)
        assert S1 == int(h.sum()) and S2 == int((h * h).sum())
        # W^2 does not depend on the height reference
        T1, T2 = oracle.width_sums(lat, H0 + 7)
        N = Lx * Ly
        assert N * S2 - S1 * S1 == N * T2 - T1 * T1


def test_width_overflow_is_reported():
    lat = oracle.flat(64, 64)
    with pytest.raises(OverflowError):
        oracle.width_sums(lat, 2**40)


@pytest.mark.parametrize("p,q", inputs.PQ_LIST)
@pytest.mark.parametrize("Lx,Ly", [(8, 8), (12, 20), (96, 64)])
def test_tiled_invariants_every_sweep(Lx, Ly, p, q):
    lat = oracle.flat(Lx, Ly)
    H0 = 0
    N = Lx * Ly
    S1_prev, _ = oracle.width_sums(lat, H0)
    c = oracle.Counts()
    for s in range(12):
        H0 = oracle.sweep(lat, p, q, seed=11, s=s, H0=H0, check=True, counts=c)
        assert_valid(lat)
        h = oracle.heights(lat, H0)
        xx, yy = np.meshgrid(np.arange(Lx), np.arange(Ly))
        assert np.all((h - xx - yy) % 2 == 0), "h = x + y (mod 2)"
        S1, S2 = oracle.width_sums(lat, H0)
        assert (S2 - S1) % 2 == 0
        assert S1 - N // 2 == 2 * (c.att - c.det), "each flip moves one height by 2"
        if q == 0.0:
            assert S1 >= S1_prev, "pure growth never lowers the mean height"
            assert c.det == 0
        if p == 0.0:
            assert c.att == 0
        S1_prev = S1


def test_rsu_invariants():
    lat = oracle.flat(16, 24)
    H0 = 0
    c = oracle.Counts()
    for t in range(10):
        H0 = oracle.rsu_sweep(lat, 0.8, 0.3, seed=5, t=t, H0=H0, counts=c)
        assert_valid(lat)
        S1, _ = oracle.width_sums(lat, H0)
        assert S1 - 16 * 24 // 2 == 2 * (c.att - c.det)


def test_identity_when_p_and_q_vanish():
    lat, H0 = inputs.rough_state(32, 32, seed=9)
    ref = lat.copy()
    H1 = oracle.run(lat, 0.0, 0.0, seed=3, t0=0, n=5, H0=H0)
    assert H1 == H0 and np.array_equal(lat, ref)
    H1 = oracle.rsu_run(lat, 0.0, 0.0, 3, 0, 2, H0)
    assert H1 == H0 and np.array_equal(lat, ref)


@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.95, 0.05), (0.3, 0.8)])
def test_mirror_symmetry_bit_for_bit(p, q):
    lat, H0 = inputs.rough_state(64, 32, seed=4)
    mir = (lat ^ 3).astype(np.uint8)
    Ha = oracle.run(lat, p, q, seed=21, t0=3, n=6, H0=H0)
    Hb = oracle.run(mir, q, p, seed=21, t0=3, n=6, H0=-H0)
    assert np.array_equal(mir, lat ^ 3)
    assert Hb == -Ha
    S1, S2 = oracle.width_sums(lat, Ha)
    T1, T2 = oracle.width_sums(mir, Hb)
    assert T1 == -S1 and T2 == S2
    # the random-sequential reference has the same symmetry
    lat2, H2 = inputs.rough_state(16, 16, seed=6)
    mir2 = (lat2 ^ 3).astype(np.uint8)
    Ha = oracle.rsu_run(lat2, p, q, 8, 0, 3, H2)
    Hb = oracle.rsu_run(mir2, q, p, 8, 0, 3, -H2)
    assert np.array_equal(mir2, lat2 ^ 3) and Hb == -Ha


def test_sweep_is_blockwise():
    """A sweep equals cutting every block out, sweeping it alone, and pasting
    it back: blocks do not communicate within a sweep (Sec. II)."""
    Lx, Ly = 96, 64
    lat, H0 = inputs.rough_state(Lx, Ly, seed=12)
    ref = lat.copy()
    seed, s, p, q = 77, 5, 0.9, 0.2
    H_ref = oracle.sweep(ref, p, q, seed, s, H0)
    Bx, By, C = oracle.geometry(Lx, Ly)
    sx, sy = oracle.block_shift(seed, s, Bx, By)
    out = lat.copy()
    dh = 0
    for j in range(Ly // By):
        for i in range(Lx // Bx):
            ys = (sy + j * By + np.arange(By)) % Ly
            xs = (sx + i * Bx + np.arange(Bx)) % Lx
            blk = np.ascontiguousarray(lat[np.ix_(ys, xs)])
            u0, v0 = (-(sx + i * Bx)) % Lx, (-(sy + j * By)) % Ly
            site00 = (u0, v0) if (u0 < Bx and v0 < By) else (-1, -1)
            d, _, _ = oracle.block_sweep(blk, C, seed, s, j * (Lx // Bx) + i, p, q, site00)
            dh += d
            out[np.ix_(ys, xs)] = blk
    assert np.array_equal(out, ref)
    assert H0 + dh == H_ref


def test_block_dead_borders_never_change():
    """The block's dead border row v = 0 and column u = 0 are never updated,
    and only they hold the bonds along that row and column, so heights along
    them, relative to the block corner, never change within a sweep."""
    Bx = By = 32
    C = 8
    blk = oracle.flat(Bx, By)
    h_before = heights_numpy(blk, 0)
    oracle.block_sweep(blk, C, seed=3, s=0, block_id=0, p=1.0, q=0.0)
    h_after = heights_numpy(blk, 0)
    # heights along row 0 and column 0 are unchanged, interior grew
    assert np.array_equal(h_after[0, :], h_before[0, :])
    assert np.array_equal(h_after[:, 0], h_before[:, 0])
    assert (h_after - h_before).sum() > 0


@pytest.mark.parametrize("Lx,Ly", inputs.SHAPES_SMALL + [(256, 256), (512, 256)])
def test_no_bond_conflicts(Lx, Ly):
    lat, H0 = inputs.rough_state(Lx, Ly, seed=2, mcs=1)
    oracle.run(lat, 0.6, 0.6, seed=1, t0=0, n=2, H0=H0, check=True)


def test_attempt_rate_per_mcs():
    """With p = q = 1 every eligible attempt flips.  Per MCS the tiled
    schedule attempts N sites minus the block borders (about 2/B of them);
    its flip count must be close to the random-sequential reference's on the
    same state (the paper's border no-ops only change prefactors, Sec. II)."""
    Lx = Ly = 256
    lat, H0 = inputs.rough_state(Lx, Ly, seed=1, mcs=2)
    a = oracle.Counts()
    b = oracle.Counts()
    oracle.run(lat.copy(), 1.0, 1.0, seed=2, t0=0, n=2, H0=H0, counts=a)
    oracle.rsu_run(lat.copy(), 1.0, 1.0, 2, 0, 2, H0, counts=b)
    ta, tb = a.att + a.det, b.att + b.det
    assert abs(ta - tb) / tb < 0.05
