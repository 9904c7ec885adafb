"""GPU parity of one-copy simulations (okpz_init_in_place) against the
oracle and against the two-copy path, bit for bit: lattice, H0 and exact width
sums for ragged sizes, every acceptance regime, both cell-border contracts,
every workgroup size, sweeps whose block segments do and do not start on a
word boundary, checkpoints, caller-owned memory, the benchmark's 2^17 x 2^17
launch and a 2^20 x 2^20 lattice (256 GiB), the size one copy makes fit."""
import numpy as np
import pytest

import oracle
from tests import inputs
from tests.test_gpu_fullsize import flat_block
from tests.test_gpu_parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def okpz():
    from paper_1110_6745_amd import okpz as m

    return m


def one_copy(okpz, Lx, Ly, p, q, seed, threads=1024, delayed=False):
    sim = okpz.okpz_init_in_place(Lx, Ly, p, q, seed)
    assert sim.copies() == 1
    sim.set_threads(threads)
    if delayed:
        sim.set_cell_borders(okpz.OKPZ_CELLS_DELAYED)
    return sim


def seed_with_aligned_sweep(Lx, Ly, within):
    """A seed whose block shift puts the segment start on a word boundary
    (sx mod 32 == 0) in one of the first `within` sweeps, and off it in another."""
    Bx, By, _ = oracle.geometry(Lx, Ly)
    for seed in range(1, 1000):
        offs = [oracle.block_shift(seed, s, Bx, By)[0] % 32 for s in range(within)]
        if 0 in offs and any(offs):
            return seed
    raise AssertionError("no seed found")


@pytest.mark.parametrize("Lx,Ly", inputs.SHAPES_GPU)
@pytest.mark.parametrize("p,q", [inputs.PQ_GROWTH, inputs.PQ_ASYM, (0.3, 0.8)])
def test_sweeps_match_oracle(okpz, Lx, Ly, p, q):
    seed = 5
    sim = one_copy(okpz, Lx, Ly, p, q, seed)
    lat, H0 = oracle.flat(Lx, Ly), 0
    for s in range(3):
        sim.sweep(1)
        H0 = oracle.sweep(lat, p, q, seed, s, H0)
        compare(sim, lat, H0, f"in place {Lx}x{Ly} p={p} q={q} after sweep {s}")
    sim.free()


@pytest.mark.parametrize("Lx,Ly", [(96, 64), (256, 256), (1056, 96)])
def test_delayed_borders_and_workgroup_sizes(okpz, Lx, Ly):
    seed = 8
    for delayed in (False, True):
        ref = oracle.flat(Lx, Ly)
        H0 = oracle.run(ref, 0.95, 0.05, seed, 0, 4, 0, delayed=delayed)
        for threads in (256, 512, 1024):
            sim = one_copy(okpz, Lx, Ly, 0.95, 0.05, seed, threads, delayed)
            sim.sweep(4)
            compare(sim, ref, H0, f"in place delayed={delayed} threads={threads}")
            sim.free()


@pytest.mark.parametrize("Lx,Ly", [(32, 64), (256, 256), (1056, 96), (4096, 32)])
def test_same_bits_as_two_copies(okpz, Lx, Ly):
    # many sweeps, including ones whose segments start on a word boundary
    # (no neighbour bits to merge) and ones that do not
    n = 40
    seed = seed_with_aligned_sweep(Lx, Ly, n)
    for p, q in [inputs.PQ_ASYM, inputs.PQ_SYM]:
        a = okpz.okpz_init(Lx, Ly, p, q, seed)
        b = one_copy(okpz, Lx, Ly, p, q, seed)
        for s in range(n):
            a.sweep(1)
            b.sweep(1)
            assert a.h0() == b.h0(), f"H0 after sweep {s}"
            if s % 8 == 7 or s == n - 1:
                assert np.array_equal(a.get_lattice(), b.get_lattice()), f"sweep {s}"
                assert a.width() == b.width(), f"width after sweep {s}"
        a.free()
        b.free()


def test_rough_start_at_large_indices(okpz):
    Lx, Ly, seed = 320, 192, 2**40 + 3
    lat, H0 = inputs.rough_state(Lx, Ly, seed=3, mcs=4)
    t0 = 2**31 + 5
    sim = one_copy(okpz, Lx, Ly, 0.9, 0.1, seed)
    sim.set_lattice(lat, H0, t0)
    ref, Hr = lat.copy(), H0
    for s in range(t0, t0 + 3):
        sim.sweep(1)
        Hr = oracle.sweep(ref, 0.9, 0.1, seed, s, Hr)
    compare(sim, ref, Hr, "in place rough start")
    sim.free()


def test_checkpoint_and_caller_memory(okpz):
    import torch

    L, seed = 128, 4
    assert okpz.okpz_required_bytes_in_place(L, L) < okpz.okpz_required_bytes(L, L)
    sim = one_copy(okpz, L, L, 0.9, 0.1, seed)
    lat, H0 = oracle.flat(L, L), 0
    sim.sweep(3)
    H0 = oracle.run(lat, 0.9, 0.1, seed, 0, 3, H0)
    back = okpz.okpz_load(sim.save())
    assert back.copies() == 1
    back.sweep(2)
    H0 = oracle.run(lat, 0.9, 0.1, seed, 3, 2, H0)
    compare(back, lat, H0, "restored one-copy run")
    back.free()
    sim.free()

    nbytes = okpz.okpz_required_bytes_in_place(L, L)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.Stream()
    with pytest.raises(okpz.OkpzError) as e:
        okpz.okpz_init_in_place(L, L, 0.9, 0.1, seed, buf.data_ptr(), nbytes - 1, stream.cuda_stream)
    assert e.value.code == okpz.OKPZ_ENOMEM
    own = okpz.okpz_init_in_place(L, L, 0.9, 0.1, seed, buf.data_ptr(), nbytes, stream.cuda_stream)
    own.sweep(5)
    compare(own, lat, H0, "one copy on caller memory")
    own.free()
    torch.cuda.synchronize()


def check_sampled_blocks(sim, L, seed, p, q, rows_j, cols_i):
    """After one sweep from the flat state: sampled blocks against the
    oracle's block update, and H0 from the block holding site (0,0)."""
    Bx, By, C = oracle.geometry(L, L)
    nbx = L // Bx
    sx, sy = oracle.block_shift(seed, 0, Bx, By)
    i00, u00 = ((L - sx) % L) // Bx, ((L - sx) % L) % Bx
    j00, v00 = ((L - sy) % L) // By, ((L - sy) % L) % By
    rows_j = sorted(set(rows_j) | {j00})
    cols_i = sorted(set(cols_i) | {i00})
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


def test_full_size_one_sweep_on_sampled_blocks(okpz):
    L, seed, p, q = 1 << 17, 1, 1.0, 0.0
    sim = one_copy(okpz, L, L, p, q, seed)
    sim.sweep(1)
    nbx = L // 256
    rng = np.random.default_rng(12)
    check_sampled_blocks(sim, L, seed, p, q, [0, nbx - 1, *rng.integers(0, nbx, 2).tolist()],
                         [0, nbx - 1, *rng.integers(0, nbx, 2).tolist()])
    sim.free()


def test_2_20_squared_fits_one_gpu(okpz):
    # 2^40 sites: one copy is 256 GiB, two would not fit in 288 GB.  The
    # sweep runs as 8 launches of 2^21 blocks; sampled blocks of the first
    # and last launch and H0 match the oracle, the width is exact.
    import torch

    torch.cuda.empty_cache()
    L, seed, p, q = 1 << 20, 2, 1.0, 0.0
    sim = one_copy(okpz, L, L, p, q, seed)
    print("allocated 2^20 x 2^20", flush=True)
    S1, S2 = sim.width(0)
    assert S1 == L * L // 2 and S2 == L * L // 2
    sim.sweep(1)
    nbx = L // 256
    check_sampled_blocks(sim, L, seed, p, q, [0, nbx // 8 - 1, nbx // 8, nbx - 1], [0, 5, nbx - 1])
    sim.free()
