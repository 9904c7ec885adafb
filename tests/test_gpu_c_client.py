"""The C ABI used from a plain C program (tests/c/okpz_c_client.c, built by
__graft_entry__.build()): sweeps, exact width, H0, the spectrum and a
checkpoint round trip, checked against the oracle."""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import psd as P
from tests.test_gpu_psd import fft_bound

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c", "okpz_c_client")


@pytest.mark.parametrize("L,p,q,seed,t", [(512, 0.95, 0.05, 7, 30), (256, 1.0, 0.0, 3, 12)])
def test_c_client_matches_oracle(L, p, q, seed, t):
    assert os.path.exists(EXE), "build the C client first (__graft_entry__.build())"
    out = subprocess.run([EXE, "run", str(L), str(p), str(q), str(seed), str(t)],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    lines = {ln.split()[0]: ln.split()[1:] for ln in out.stdout.strip().splitlines()}
    lat = oracle.flat(L, L)
    H0 = oracle.run(lat, p, q, seed, 0, t, 0)
    S1, S2 = oracle.width_sums(lat, H0)
    assert [int(v) for v in lines["width"]] == [t, S1, S2, H0]
    h = oracle.heights(lat, H0)
    Sx, Sy = P.psd_axes(h)
    got = [float(v) for v in lines["psd"]]
    want = [Sx[1], Sy[1], Sx[2], Sy[2]]
    # the spectrum tests' bound (radix-2 FFTs of the profile and of the
    # oracle's N heights, fp64)
    N = L * L
    d_or = fft_bound(N, float(np.linalg.norm(h - h.mean())))
    for g, w, prof in zip(got, want, (h.sum(axis=0), h.sum(axis=1)) * 2):
        delta = d_or + fft_bound(L, float(np.linalg.norm(prof - prof.mean())))
        assert abs(g - w) <= (2 * math.sqrt(N * w) + delta) * delta / N, (got, want)
    assert "restore" in lines
