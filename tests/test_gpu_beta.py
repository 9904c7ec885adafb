"""The beta judge: the tiled GPU dynamics against the random-sequential
reference in the effective growth exponent.

Sec. II expects the decomposition of the lattice into blocks and thread cells
to change prefactors of the width but not exponents; Sec. III measures the
growth exponent through beta_eff(t), the discretised log-derivative of W(t)
with t/t' = 2 (Eq. (beff)), after subtracting the flat state's intrinsic
width 1/4 and leaving out t < t_mic ~ 50.

The random-sequential side is the oracle's ensemble stored under
tests/golden/ by tests/golden/make_rsu_growth.py (L = 1024, p = 1, q = 0,
32 seeds, widths at the Sec. III times with m = 0.01 up to t = 4096).  The
GPU side runs both cell-border contracts of the tiled dynamics through one
persistent batch launch each, 64 seeds, same L, p, q and times.  Errors are
delete-one jackknife errors over seeds on each side, combined in quadrature;
the test requires every window and the mean over windows to agree within
3 combined standard errors, with no other slack.
"""
import os

import numpy as np
import pytest

from tests import beta as B

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "rsu_growth_L1024_p1_q0.txt")
TARGETS = [64 * 2**k for k in range(7)]  # t' = 64 > t_mic up to t = 4096
R_GPU, SEED0_GPU = 64, 20001


def load_gold(path):
    params, rows = {}, []
    with open(path) as f:
        for line in f:
            if line.startswith("# L "):
                tok = line[2:].split()
                params = {tok[i]: tok[i + 1] for i in range(0, len(tok), 2)}
            elif not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    a = np.array(rows, dtype=object)
    seeds = sorted(set(a[:, 0].tolist()))
    times = sorted(set(a[:, 1].tolist()))
    S = {(r[0], r[1]): (r[2], r[3]) for r in rows}
    return params, seeds, times, S


@pytest.fixture(scope="module")
def okpz():
    from paper_1110_6745_amd import okpz as m

    return m


def test_beta_eff_matches_random_sequential(okpz):
    params, seeds, times, S = load_gold(GOLD)
    L, p, q = int(params["L"]), float(params["p"]), float(params["q"])
    t_max, m = int(params["t_max"]), float(params["m"])
    N = L * L
    assert times == okpz.sampling_times(t_max, m)
    tk = B.pick_times(times, TARGETS)
    w_rsu = np.array([[B.excess_w2([S[(s, t)][0]], [S[(s, t)][1]], N)[0] for t in tk]
                      for s in seeds])
    b_rsu, c_rsu = B.jackknife(w_rsu, tk)

    result = {}
    for kind, name in ((okpz.OKPZ_CELLS_DEAD, "dead"), (okpz.OKPZ_CELLS_DELAYED, "delayed")):
        jobs = [(L, L, p, q, SEED0_GPU + r, t_max) for r in range(R_GPU)]
        b = okpz.Batch(jobs, m)
        b.set_cell_borders(kind)
        ms = b.run()
        w = np.zeros((R_GPU, len(tk)))
        for r in range(R_GPU):
            t, s1, s2 = b.samples(r)
            assert t.tolist() == times
            pos = [times.index(x) for x in tk]
            w[r] = B.excess_w2([int(s1[i]) for i in pos], [int(s2[i]) for i in pos], N)
        b.free()
        print(f"\n{name}: {R_GPU} x {L}^2 to t = {t_max} in {ms / 1e3:.2f} s", flush=True)
        result[name] = (w, B.jackknife(w, tk))

    print(f"\nbeta_eff, L = {L}, p = {p}, q = {q}; t' -> t (t/t' ~ 2), jackknife errors")
    print("  t' ->    t " + "".join(f"{'rsu':>16s}{'dead':>16s}{'delayed':>16s}"))
    for k in range(len(tk) - 1):
        row = f"{tk[k]:5d} -> {tk[k + 1]:4d} {b_rsu[k]:9.4f}({np.sqrt(c_rsu[k, k]):.4f})"
        for name in ("dead", "delayed"):
            bb, cc = result[name][1]
            row += f" {bb[k]:9.4f}({np.sqrt(cc[k, k]):.4f})"
        print(row)
    mean_w = {"rsu": w_rsu.mean(axis=0)}
    for name in ("dead", "delayed"):
        mean_w[name] = result[name][0].mean(axis=0)
    print("excess W^2 at t: " + " ".join(f"{t}" for t in tk))
    for name, v in mean_w.items():
        print(f"  {name:8s} " + " ".join(f"{x:.4f}" for x in v))

    K = len(tk) - 1
    for name in ("dead", "delayed"):
        bb, cc = result[name][1]
        d = bb - b_rsu
        sig = np.sqrt(np.diag(cc) + np.diag(c_rsu))
        z = d / sig
        dbar = d.mean()
        sbar = np.sqrt((cc + c_rsu).sum()) / K
        print(f"{name} - rsu in combined standard errors: " + " ".join(f"{v:+.2f}" for v in z)
              + f"; mean over windows {dbar:+.4f} +- {sbar:.4f}")
        assert np.all(np.abs(z) < 3.0), f"{name}: beta_eff differs from the reference"
        assert abs(dbar) < 3.0 * sbar, f"{name}: mean beta_eff differs from the reference"
