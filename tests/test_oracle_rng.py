"""Pins of the oracle's random numbers and constants (CPU only).

The counter-based generator replaces the paper's per-thread LCRNGs (Sec. II)
so that a trajectory is a pure function of the seed; these tests fix it
against published known answers and an independent implementation.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], tuple(v[6:10])))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert oracle.philox(ctr, key) == want


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    exe = str(tmp_path_factory.mktemp("probe") / "rocrand_philox_probe")
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", os.path.join(HERE, "rocrand_philox_probe.cpp"),
                    "-o", exe], check=True)
    return exe


def test_philox_matches_rocrand(rocrand_probe):
    rng = np.random.default_rng(1234)
    q = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    # include the counter shapes the dynamics uses
    q[0] = [5, 0, 0, 2, 1, 0]
    q[1] = [7, 1000, (3 << 16) | 1023, 0, 0xDEADBEEF, 42]
    inp = "\n".join(" ".join(f"{int(v):x}" for v in row) for row in q) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for row, line in zip(q, out):
        want = tuple(int(t, 16) for t in line.split())
        assert oracle.philox(row[:4], row[4:]) == want


def test_philox_output_is_balanced():
    # 4096 outputs of consecutive counters: every bit is set about half the time
    words = np.array([oracle.philox([i, 0, 0, 0], [7, 0]) for i in range(1024)],
                     dtype=np.uint64).ravel()
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint64)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.04)


def test_threshold_endpoints_and_rounding():
    assert oracle.threshold(0.0) == 0
    assert oracle.threshold(1.0) == 2**32
    assert oracle.threshold(0.5) == 2**31
    assert oracle.threshold(0.25) == 2**30
    assert oracle.threshold(-0.1) == 0
    assert oracle.threshold(1.5) == 2**32
    assert oracle.threshold(float("nan")) == 0
    # round half away from zero of p * 2^32
    assert oracle.threshold(0.95) == round(0.95 * 2**32)
    assert oracle.threshold(1.0 / 3.0) == int(np.floor((1.0 / 3.0) * 2**32 + 0.5))
    ts = [oracle.threshold(p) for p in np.linspace(0, 1, 101)]
    assert all(a <= b for a, b in zip(ts, ts[1:]))


@pytest.mark.parametrize("L,B", [(4, 4), (12, 4), (32, 32), (96, 32), (256, 256),
                                 (4096, 256), (2**17, 256), (1000, 8), (768, 256)])
def test_geometry(L, B):
    Bx, By, C = oracle.geometry(L, L)
    assert Bx == B and By == B
    assert C == min(8, B)
    assert L % Bx == 0


def test_geometry_rejects_bad_sizes():
    for Lx, Ly in [(2, 4), (6, 8), (4, 10), (0, 4)]:
        with pytest.raises(ValueError):
            oracle.geometry(Lx, Ly)


def test_block_shift_uniform():
    # shifts over many sweeps cover [0,B) x [0,B) evenly
    B = 8
    cnt = np.zeros((B, B))
    for s in range(6400):
        sx, sy = oracle.block_shift(99, s, B, B)
        assert 0 <= sx < B and 0 <= sy < B
        cnt[sy, sx] += 1
    chi2 = ((cnt - 100.0) ** 2 / 100.0).sum()
    assert chi2 < 130  # 63 dof; p ~ 1e-6 threshold
