"""okpz_psd_noalloc: the spectrum (Sec. III, Eqs. (PSD), (hF)) without any
device allocation, on the library's fixed per-GPU scratch.

Checked through the C ABI against okpz_psd, the entry point it varies, bit
for bit (both run the same kernels; the column counts are exact integers
whatever the chunking, and the transforms see identical inputs), on calls in
a row with inputs that shrink, so nothing left in the shared scratch by one
call can reach the next: the largest lattice it takes (2^17 x 2^17, where the
static scratch forces taller column-count chunks than okpz_psd uses), then a
lattice with a Bluestein side, then a small one.  The last two are also held
to the oracle's fft2 of the heights within the fp64 FFT bound of the
spectrum parity tests.  A side above 2^17 is rejected, and a call leaves the
device's free memory unchanged.
"""
import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def okpz():
    from paper_1110_6745_amd import okpz as m

    return m


def same(a, b):
    return all(np.array_equal(x.view(np.uint64), y.view(np.uint64)) for x, y in zip(a, b))


def test_noalloc_spectrum_equals_okpz_psd_on_shrinking_inputs(okpz):
    import torch

    from tests.test_gpu_psd import check

    L = 1 << 17
    big = okpz.okpz_init(L, L, 1.0, 0.0, 5)
    big.sweep(3)
    first = big.psd_noalloc()
    assert same(first, big.psd()), "2^17 x 2^17: okpz_psd_noalloc differs from okpz_psd"
    free0 = torch.cuda.mem_get_info()[0]
    again = big.psd_noalloc()
    assert torch.cuda.mem_get_info()[0] == free0, "okpz_psd_noalloc changed free device memory"
    assert same(first, again)
    big.free()
    print("2^17 x 2^17 ok", flush=True)

    for (Lx, Ly), seed in (((2048, 1056), 11), ((256, 96), 12)):
        lat, H0 = inputs.rough_state(Lx, Ly, seed=seed, mcs=4)
        sim = okpz.okpz_init(Lx, Ly, 0.95, 0.05, seed)
        sim.set_lattice(lat, H0, 0)
        got = sim.psd_noalloc()
        assert same(got, sim.psd()), f"{Lx}x{Ly}: okpz_psd_noalloc differs from okpz_psd"
        check(got, lat, H0, f"{Lx}x{Ly} noalloc")
        sim.free()
        print(f"{Lx}x{Ly} ok", flush=True)


def test_noalloc_spectrum_rejects_sides_beyond_its_scratch(okpz):
    sim = okpz.okpz_init(1 << 18, 32, 1.0, 0.0, 1)
    with pytest.raises(okpz.OkpzError) as e:
        sim.psd_noalloc()
    assert e.value.code == okpz.OKPZ_EINVAL and "static scratch" in str(e.value)
    sim.free()
