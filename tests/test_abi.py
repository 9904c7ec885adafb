"""The C-ABI library loads and exports every symbol ``include/okpz.h``
declares; argument validation that happens before any device call (CPU)."""
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "okpz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(okpz_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1110_6745_amd import okpz

    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(okpz.lib(), n), f"{n} not exported"
    assert sorted(okpz.EXPORTED) == names


def test_geometry_matches_oracle():
    from paper_1110_6745_amd import okpz

    for Lx, Ly in [(32, 32), (96, 64), (256, 256), (320, 192), (4096, 4096), (2**17, 2**17),
                   (1024, 32)]:
        assert okpz.okpz_geometry(Lx, Ly) == oracle.geometry(Lx, Ly)


def test_required_bytes():
    from paper_1110_6745_amd import okpz

    # two lattice copies of 2 bits per site + small scratch
    n = okpz.okpz_required_bytes(2**17, 2**17)
    assert 2 * 2**34 // 4 <= n < 2 * 2**34 // 4 + 2**22
    assert okpz.okpz_required_bytes(33, 32) == 0


def test_required_bytes_in_place():
    from paper_1110_6745_amd import okpz

    # one lattice copy: exactly one copy's bytes less than two copies, and the
    # largest lattice, 2^20 x 2^20, within 256 GiB + 64 MiB
    for Lx, Ly in [(32, 32), (96, 64), (2**17, 2**17), (2**20, 2**20)]:
        one, two = okpz.okpz_required_bytes_in_place(Lx, Ly), okpz.okpz_required_bytes(Lx, Ly)
        plane = -(-(Lx * Ly // 4) // 256) * 256
        assert two - one == plane
    assert okpz.okpz_required_bytes_in_place(2**20, 2**20) < 2**38 + 2**26
    assert okpz.okpz_required_bytes_in_place(32, 48) == 0


@pytest.mark.parametrize("Lx,Ly,p,q", [(33, 32, 1, 0), (32, 2**21, 1, 0), (32, 32, 0, 2.0)])
def test_init_in_place_rejects_bad_arguments(Lx, Ly, p, q):
    # rejected on the host before any device call
    from paper_1110_6745_amd import okpz

    with pytest.raises(okpz.OkpzError) as e:
        okpz.okpz_init_in_place(Lx, Ly, p, q, 1)
    assert e.value.code == okpz.OKPZ_EINVAL


@pytest.mark.parametrize("Lx,Ly,p,q", [(33, 32, 1, 0), (32, 16, 1, 0), (0, 32, 1, 0),
                                        (2**21, 32, 1, 0), (32, 32, 1.5, 0), (32, 32, 0, -0.1),
                                        (32, 32, float("nan"), 0)])
def test_init_rejects_bad_arguments(Lx, Ly, p, q):
    from paper_1110_6745_amd import okpz

    with pytest.raises(okpz.OkpzError) as e:
        okpz.okpz_init(Lx, Ly, p, q, 1)
    assert e.value.code == okpz.OKPZ_EINVAL


@pytest.mark.parametrize("job,m", [((33, 32, 1, 0, 1, 5), 0.01), ((32, 32, 1.2, 0, 1, 5), 0.01),
                                   ((32, 32, 1, 0, 1, -1), 0.01), ((32, 32, 1, 0, 1, 5), 0.0),
                                   ((16384, 32, 1, 0, 1, 5), 0.01)])
def test_batch_rejects_bad_jobs(job, m):
    from paper_1110_6745_amd import okpz

    with pytest.raises(okpz.OkpzError) as e:
        okpz.Batch([job], m)
    assert e.value.code == okpz.OKPZ_EINVAL


def test_sampling_times_follow_the_paper_recurrence():
    from paper_1110_6745_amd import okpz

    # t_{i+1} = (t_i + 10) e^m from t_0 = 0 (Sec. III), rounded up
    assert okpz.sampling_times(100, 0.01)[:4] == [11, 21, 31, 42]
    assert okpz.sampling_times(100, 0.01)[-1] == 100
    assert okpz.sampling_times(0, 0.01) == []


def test_header_is_c99_and_host_calls_work_from_c(tmp_path):
    # a plain C client compiled as strict C99 against include/okpz.h and
    # linked with the library; its host-only calls run without a GPU
    import subprocess

    exe = str(tmp_path / "client")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "okpz_c_client.c"),
                    "-L", os.path.join(ROOT, "paper_1110_6745_amd"), "-lokpz",
                    "-Wl,-rpath," + os.path.join(ROOT, "paper_1110_6745_amd"), "-o", exe],
                   check=True)
    out = subprocess.run([exe, "host"], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "host ok"


@pytest.mark.parametrize("m", [0.001, 0.01, 0.0663, 0.5, 3.0, 10.0])
def test_sampling_times_equal_the_oracle(m):
    # the library's one implementation against the oracle's own
    from paper_1110_6745_amd import okpz

    for t_max in (0, 1, 9, 11, 100, 4096, 10000, 1_310_720):
        assert okpz.sampling_times(t_max, m) == oracle.sampling_times(t_max, m), (t_max, m)


@pytest.mark.parametrize("t_max,m", [(100, 0.0), (100, -0.1), (100, 10.5), (-1, 0.01),
                                     (1 << 32, 0.01), (100, float("nan"))])
def test_sampling_times_reject_bad_arguments(t_max, m):
    from paper_1110_6745_amd import okpz

    with pytest.raises(okpz.OkpzError) as e:
        okpz.sampling_times(t_max, m)
    assert e.value.code == okpz.OKPZ_EINVAL


def _flat_checkpoint(Lx=64, Ly=32, H0=0, ox=0, t=5):
    """A checkpoint of the flat state: the 80-byte header of include/okpz.h's
    okpz_save layout, then the sigma_x and sigma_y bit planes."""
    import struct

    import numpy as np

    hdr = struct.pack("<8sIIqqddQqqii", b"OKPZCKP1", 1, 0, Lx, Ly, 1.0, 0.0, 7, t, H0, ox, 2)
    assert len(hdr) == 80
    W = Lx // 32
    rows = np.array([0x55555555 if y % 2 == 0 else 0xAAAAAAAA for y in range(Ly)], np.uint32)
    plane = np.repeat(rows, W)
    return bytearray(hdr + plane.tobytes() + plane.tobytes())


def _load_code(buf):
    from paper_1110_6745_amd import okpz

    try:
        sim = okpz.okpz_load(bytes(buf))
    except okpz.OkpzError as e:
        return e.code
    sim.free()  # a device was there and the checkpoint loaded
    return okpz.OKPZ_OK


def test_load_rejects_corrupt_checkpoints_before_any_device_call():
    from paper_1110_6745_amd import okpz

    good = _flat_checkpoint()
    # the valid checkpoint passes validation (on a host without a device the
    # allocation that follows fails instead)
    assert _load_code(good) != okpz.OKPZ_EINVAL
    bad = bytearray(good)
    bad[0:8] = b"OKPZCKP2"
    assert _load_code(bad) == okpz.OKPZ_EINVAL
    assert _load_code(good[:-1]) == okpz.OKPZ_EINVAL           # truncated planes
    assert _load_code(good[:40]) == okpz.OKPZ_EINVAL           # truncated header
    assert _load_code(_flat_checkpoint(H0=3)) == okpz.OKPZ_EINVAL  # odd h(0,0)
    assert _load_code(_flat_checkpoint(ox=64)) == okpz.OKPZ_EINVAL
    assert _load_code(_flat_checkpoint(Lx=48)) == okpz.OKPZ_EINVAL
    assert _load_code(_flat_checkpoint(t=-1)) == okpz.OKPZ_EINVAL
    # one flipped slope bit opens two plaquettes and breaks a row sum
    bad = bytearray(good)
    bad[80 + 4 * 5] ^= 0x10
    assert _load_code(bad) == okpz.OKPZ_EINVAL
    # one flipped sigma_y bit
    bad = bytearray(good)
    bad[80 + 64 * 32 // 8 + 9] ^= 0x01
    assert _load_code(bad) == okpz.OKPZ_EINVAL
    # a rotated valid field (stored columns shifted) is still valid
    assert _load_code(_flat_checkpoint(ox=17)) != okpz.OKPZ_EINVAL
