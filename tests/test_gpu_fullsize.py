"""GPU parity at the benchmark's full size and at the other workload sizes.

* 2^17 x 2^17 (the benchmark's launch configuration): flat state width in
  closed form (Sec. III, W^2 = 1/4); one sweep from the flat state checked
  block by block against the oracle on sampled blocks (blocks are
  independent within a sweep, Sec. II), including the block holding site
  (0,0), so H0 is checked too; q = 0 growth never lowers sum h.
* 4096 x 4096, both (p, q) of the medium workload, whole-lattice parity for
  a few MCS.
* Rows of full length 2^17 and columns of full height 2^17 for the width
  path, on oracle-made rough states.
* A 2^19 x 2^19 lattice, whose sweep is split over two launches, on
  sampled blocks; the longest sides taken (2^20 x 32, 32 x 2^20) whole.
"""
import numpy as np
import pytest

import oracle
from tests import inputs

pytestmark = pytest.mark.gpu

L17 = 1 << 17


@pytest.fixture(scope="module")
def okpz():
    from paper_1110_6745_amd import okpz as m

    return m


def flat_block(x0, y0, Bx, By):
    """Cut-out of the flat state at (x0, y0); the flat state has period 2."""
    big = oracle.flat(Bx + 2, By + 2)
    return np.ascontiguousarray(big[y0 % 2: y0 % 2 + By, x0 % 2: x0 % 2 + Bx])


def test_full_size_flat_width_and_one_sweep(okpz):
    L = L17
    N = L * L
    seed, p, q = 1, 1.0, 0.0
    sim = okpz.okpz_init(L, L, p, q, seed)
    S1, S2 = sim.width(0)
    assert S1 == N // 2 and S2 == N // 2 and 4 * (N * S2 - S1 * S1) == N * N
    print("flat width ok", flush=True)
    sim.sweep(1)
    Bx, By, C = oracle.geometry(L, L)
    nbx = L // Bx
    sx, sy = oracle.block_shift(seed, 0, Bx, By)
    i00, u00 = ((L - sx) % L) // Bx, ((L - sx) % L) % Bx
    j00, v00 = ((L - sy) % L) // By, ((L - sy) % L) % By
    rng = np.random.default_rng(5)
    rows_j = sorted({0, 1, j00, nbx - 1, *rng.integers(0, nbx, 2).tolist()})
    cols_i = sorted({0, 1, i00, nbx - 1, *rng.integers(0, nbx, 3).tolist()})
    dh_total = 0
    for j in rows_j:
        y0 = (sy + j * By) % L
        got_rows = sim.get_rows(y0, By)  # (By, L) canonical bytes
        for i in cols_i:
            x0 = (sx + i * Bx) % L
            blk = flat_block(x0, y0, Bx, By)
            site00 = (u00, v00) if (i == i00 and j == j00) else (-1, -1)
            dh, att, det = oracle.block_sweep(blk, C, seed, 0, j * nbx + i, p, q, site00)
            dh_total += dh
            xs = (x0 + np.arange(Bx)) % L
            assert np.array_equal(got_rows[:, xs], blk), f"block ({i},{j}) differs"
        print(f"block row {j} ok", flush=True)
    assert sim.h0() == dh_total
    S1b, _ = sim.width(1)
    sim.sweep(2)
    S1c, _ = sim.width(3)
    assert N // 2 < S1b <= S1c, "pure growth never lowers the mean height"
    sim.free()


@pytest.mark.parametrize("p,q", [inputs.PQ_GROWTH, inputs.PQ_ASYM])
def test_medium_workload_whole_lattice(okpz, p, q):
    L, seed = 4096, 1
    sim = okpz.okpz_init(L, L, p, q, seed)
    lat = oracle.flat(L, L)
    H0 = 0
    for t in (1, 3):
        H0 = oracle.run(lat, p, q, seed, sim.time(), t - sim.time(), H0)
        assert sim.width(t) == oracle.width_sums(lat, H0), f"t={t}"
    assert np.array_equal(sim.get_lattice(), lat)
    assert sim.h0() == H0
    sim.free()


@pytest.mark.parametrize("Lx,Ly", [(L17, 64), (64, L17)])
def test_full_length_rows_and_columns(okpz, Lx, Ly):
    lat, H0 = inputs.rough_state(Lx, Ly, seed=31, mcs=2)
    sim = okpz.okpz_init(Lx, Ly, 0.95, 0.05, 3)
    sim.set_lattice(lat, H0, 0)
    assert sim.width() == oracle.width_sums(lat, H0)
    sim.sweep(2)
    H1 = oracle.run(lat, 0.95, 0.05, 3, 0, 2, H0)
    assert sim.width() == oracle.width_sums(lat, H1)
    assert np.array_equal(sim.get_lattice(), lat) and sim.h0() == H1
    sim.free()


def test_sweep_split_over_launches_at_2_19(okpz):
    # 2^19 x 2^19 (128 GiB for both copies) has 2^22 blocks of 256^2, more
    # work-items than one grid dimension holds: the sweep runs as two
    # launches; sampled blocks of both halves and H0 match the oracle
    L = 1 << 19
    seed, p, q = 3, 1.0, 0.0
    sim = okpz.okpz_init(L, L, p, q, seed)
    sim.sweep(1)
    Bx, By, C = oracle.geometry(L, L)
    nbx = L // Bx
    sx, sy = oracle.block_shift(seed, 0, Bx, By)
    i00, u00 = ((L - sx) % L) // Bx, ((L - sx) % L) % Bx
    j00, v00 = ((L - sy) % L) // By, ((L - sy) % L) % By
    rows_j = sorted({0, j00, nbx // 2 - 1, nbx // 2, nbx - 1})
    cols_i = sorted({0, i00, 7, nbx - 1})
    dh_total = 0
    for j in rows_j:
        y0 = (sy + j * By) % L
        got_rows = sim.get_rows(y0, By)
        for i in cols_i:
            x0 = (sx + i * Bx) % L
            blk = flat_block(x0, y0, Bx, By)
            site00 = (u00, v00) if (i == i00 and j == j00) else (-1, -1)
            dh, _, _ = oracle.block_sweep(blk, C, seed, 0, j * nbx + i, p, q, site00)
            dh_total += dh
            xs = (x0 + np.arange(Bx)) % L
            assert np.array_equal(got_rows[:, xs], blk), f"block ({i},{j}) differs"
        print(f"block row {j} ok", flush=True)
    assert sim.h0() == dh_total
    sim.free()


@pytest.mark.parametrize("Lx,Ly", [(1 << 20, 32), (32, 1 << 20)])
def test_longest_sides(okpz, Lx, Ly):
    # the largest side the library takes (2^20) against the smallest (32):
    # sweeps, exact width and the spectrum (a 2^20-point transform)
    from oracle import psd as P
    from tests.test_gpu_psd import check

    lat, H0 = inputs.rough_state(Lx, Ly, seed=41, mcs=1)
    sim = okpz.okpz_init(Lx, Ly, 0.9, 0.15, 41)
    sim.set_lattice(lat, H0, 7)
    sim.sweep(3)
    H1 = oracle.run(lat, 0.9, 0.15, 41, 7, 3, H0)
    assert sim.width() == oracle.width_sums(lat, H1)
    assert np.array_equal(sim.get_lattice(), lat) and sim.h0() == H1
    check(sim.psd(), lat, H1, f"{Lx}x{Ly}")
    sim.free()
