"""GPU parity: the HIP path (through the C ABI) against the oracle, bit for bit.

Lattices, the absolute height H0 and the exact int64 width sums must be
identical after every checked sweep, for square and ragged sizes (block sides
32 .. 256, several blocks plus a ragged count), every (p, q) regime, rough
start states produced by the oracle, and large sweep indices and seeds.
"""
import numpy as np
import pytest

import oracle
from tests import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def okpz():
    from paper_1110_6745_amd import okpz as m

    return m


def compare(sim, lat, H0, what):
    got = sim.get_lattice()
    if not np.array_equal(got, lat):
        bad = np.argwhere(got != lat)
        raise AssertionError(f"{what}: {len(bad)} sites differ, first at (y,x)={tuple(bad[0])}")
    assert sim.h0() == H0, f"{what}: H0 {sim.h0()} != {H0}"
    assert sim.width() == oracle.width_sums(lat, H0), f"{what}: width sums differ"


def test_flat_state(okpz):
    for Lx, Ly in [(32, 32), (96, 64), (256, 256), (4096, 32)]:
        sim = okpz.okpz_init(Lx, Ly, 1.0, 0.0, 1)
        lat = oracle.flat(Lx, Ly)
        compare(sim, lat, 0, f"flat {Lx}x{Ly}")
        N = Lx * Ly
        S1, S2 = sim.width(0)
        assert S1 == N // 2 and S2 == N // 2 and 4 * (N * S2 - S1 * S1) == N * N
        assert abs(sim.w2() - 0.25) < 1e-15
        sim.free()


@pytest.mark.parametrize("Lx,Ly", inputs.SHAPES_GPU)
@pytest.mark.parametrize("p,q", inputs.PQ_LIST[:5])
def test_sweeps_match_oracle(okpz, Lx, Ly, p, q):
    seed = 1 + Lx + 7 * Ly
    sim = okpz.okpz_init(Lx, Ly, p, q, seed)
    lat = oracle.flat(Lx, Ly)
    H0 = 0
    for s in range(6):
        sim.sweep(1)
        H0 = oracle.sweep(lat, p, q, seed, s, H0)
        compare(sim, lat, H0, f"{Lx}x{Ly} p={p} q={q} after sweep {s}")
    sim.free()


@pytest.mark.parametrize("Lx,Ly,seed", [(64, 96, 3), (256, 256, 2**40 + 17), (512, 1024, 5)])
def test_rough_start_and_large_indices(okpz, Lx, Ly, seed):
    lat, H0 = inputs.rough_state(Lx, Ly, seed=seed % 1000, mcs=4)
    t0 = 2**31 + 11
    for p, q in [(0.95, 0.05), (0.3, 0.8)]:
        sim = okpz.okpz_init(Lx, Ly, p, q, seed)
        sim.set_lattice(lat, H0, t0)
        ref = lat.copy()
        Hr = H0
        for s in range(t0, t0 + 3):
            sim.sweep(1)
            Hr = oracle.sweep(ref, p, q, seed, s, Hr)
        compare(sim, ref, Hr, f"rough {Lx}x{Ly} seed={seed} p={p}")
        sim.free()


def test_identity_and_mirror(okpz):
    Lx, Ly = 128, 96
    lat, H0 = inputs.rough_state(Lx, Ly, seed=8)
    sim = okpz.okpz_init(Lx, Ly, 0.0, 0.0, 9)
    sim.set_lattice(lat, H0, 0)
    sim.sweep(3)
    compare(sim, lat, H0, "p=q=0 identity")
    sim.free()
    a = okpz.okpz_init(Lx, Ly, 0.9, 0.2, 4)
    b = okpz.okpz_init(Lx, Ly, 0.2, 0.9, 4)
    a.set_lattice(lat, H0, 0)
    b.set_lattice(lat ^ 3, -H0, 0)
    a.sweep(4)
    b.sweep(4)
    assert np.array_equal(a.get_lattice() ^ 3, b.get_lattice())
    assert a.h0() == -b.h0()
    a.free()
    b.free()


def test_small_workload_full(okpz):
    """256 x 256, p = 1, q = 0, seed 1, 100 MCS, widths at the sampling
    times t_{i+1} = (t_i + 10) e^m with m = 0.01 (Sec. III), rounded up."""
    Lx = Ly = 256
    sim = okpz.okpz_init(Lx, Ly, 1.0, 0.0, 1)
    lat = oracle.flat(Lx, Ly)
    H0 = 0
    times, t = [], 0.0
    while True:
        t = (t + 10.0) * np.exp(0.01)
        if t > 100:
            break
        times.append(int(np.ceil(t)))
    times = sorted(set(times)) + [100]
    now = 0
    for T in times:
        H0 = oracle.run(lat, 1.0, 0.0, 1, now, T - now, H0)
        now = T
        assert sim.width(T) == oracle.width_sums(lat, H0), f"t={T}"
    compare(sim, lat, H0, "256^2 after 100 MCS")
    sim.free()


def test_checkpoint_resume_is_bit_exact(okpz):
    Lx, Ly = 192, 128
    a = okpz.okpz_init(Lx, Ly, 0.95, 0.05, 77)
    a.sweep(5)
    blob = a.save()
    a.sweep(4)
    b = okpz.okpz_load(blob)
    assert b.time() == 5
    b.sweep(4)
    assert np.array_equal(a.get_lattice(), b.get_lattice())
    assert a.h0() == b.h0() and a.width() == b.width()
    a.free()
    b.free()


def test_errors(okpz):
    sim = okpz.okpz_init(64, 64, 1.0, 0.0, 1)
    sim.sweep(3)
    with pytest.raises(okpz.OkpzError) as e:
        sim.width(2)
    assert e.value.code == okpz.OKPZ_EINVAL
    bad = oracle.flat(64, 64)
    bad[3, 5] ^= 1  # breaks a row sum
    with pytest.raises(okpz.OkpzError):
        sim.set_lattice(bad, 0, 0)
    # h = x + y (mod 2): the height of site (0,0) is even
    with pytest.raises(okpz.OkpzError) as e:
        sim.set_lattice(oracle.flat(64, 64), 7, 0)
    assert e.value.code == okpz.OKPZ_EINVAL
    sim.set_lattice(oracle.flat(64, 64), 2**40, 0)
    with pytest.raises(okpz.OkpzError) as e:
        sim.width()
    assert e.value.code == okpz.OKPZ_EOVERFLOW
    sim.free()


def test_init_on_caller_buffer_and_stream(okpz):
    import torch

    Lx, Ly = 256, 128
    n = okpz.okpz_required_bytes(Lx, Ly)
    buf = torch.empty(n, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    sim = okpz.okpz_init_on(Lx, Ly, 1.0, 0.0, 3, buf.data_ptr(), n, st.cuda_stream)
    sim.sweep(3)
    ref = oracle.flat(Lx, Ly)
    H0 = oracle.run(ref, 1.0, 0.0, 3, 0, 3, 0)
    compare(sim, ref, H0, "init_on")
    sim.free()
    del buf


@pytest.mark.parametrize("Lx,Ly", [(256, 256), (96, 64), (512, 256), (1056, 96), (2080, 64)])
def test_execution_mapping_does_not_change_the_result(okpz, Lx, Ly):
    """Every workgroup size gives the same bits (the contract keys random
    decisions by cell, never by thread); also a race detector for the LDS
    step loop."""
    ref = oracle.flat(Lx, Ly)
    H0 = oracle.run(ref, 0.95, 0.05, 6, 0, 4, 0)
    for threads in (256, 512, 1024):
        sim = okpz.okpz_init(Lx, Ly, 0.95, 0.05, 6)
        sim.set_threads(threads)
        sim.sweep(4)
        compare(sim, ref, H0, f"threads={threads}")
        sim.free()


@pytest.mark.parametrize("p,q", [inputs.PQ_GROWTH, inputs.PQ_ASYM])
def test_every_sweep_for_a_hundred_sweeps(okpz, p, q):
    """One 256 x 256 block, 100 sweeps, lattice and H0 checked after every
    sweep (the block containing site (0,0) is the whole lattice, so every
    sweep exercises the H0 bookkeeping)."""
    Lx = Ly = 256
    sim = okpz.okpz_init(Lx, Ly, p, q, 1)
    lat = oracle.flat(Lx, Ly)
    H0 = 0
    for s in range(100):
        sim.sweep(1)
        H0 = oracle.sweep(lat, p, q, 1, s, H0)
        assert sim.h0() == H0, f"sweep {s}: H0 {sim.h0()} != {H0}"
        if s % 10 == 9:
            assert np.array_equal(sim.get_lattice(), lat), f"sweep {s}: lattice differs"
    sim.free()
