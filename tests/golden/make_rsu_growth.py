"""Write the random-sequential growth ensemble the beta_eff comparison reads.

Calls only ``oracle``: R flat-start realizations (Sec. III) of the textbook
random-sequential dynamics of Eq. (1) on an L x L torus, with the exact width
sums (S1, S2) = (sum h, sum h^2) at the measurement times of Sec. III
(t_{i+1} = (t_i + 10) e^m, m = 0.01) up to t_max.

    python tests/golden/make_rsu_growth.py [L] [p] [q] [R] [t_max] [seed0]

writes ``tests/golden/rsu_growth_L{L}_p{p}_q{q}.txt``: '#' header lines with
the parameters, then one line per (seed, time): ``seed t S1 S2``.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main(L=1024, p=1.0, q=0.0, R=32, t_max=4096, seed0=9001, m=0.01):
    times = oracle.sampling_times(t_max, m)
    t0 = time.time()
    ens = oracle.ensemble_at(L, L, p, q, seed0, R, times, rsu=True)
    dt = time.time() - t0
    path = os.path.join(HERE, f"rsu_growth_L{L}_p{p:g}_q{q:g}.txt")
    with open(path, "w") as f:
        f.write("# random-sequential reference (oracle.ensemble_at, rsu=True), flat start\n")
        f.write(f"# L {L} p {p!r} q {q!r} R {R} seed0 {seed0} t_max {t_max} m {m!r}\n")
        f.write(f"# oracle threads {oracle.num_threads()}, {dt:.0f} s\n")
        f.write("# seed t S1 S2\n")
        for r in range(R):
            for i, t in enumerate(times):
                f.write(f"{seed0 + r} {t} {ens[r, i, 0]} {ens[r, i, 1]}\n")
    print(path, f"{dt:.0f} s")


if __name__ == "__main__":
    a = sys.argv[1:]
    kw = {}
    names = ["L", "p", "q", "R", "t_max", "seed0"]
    conv = [int, float, float, int, int, int]
    for n, c, v in zip(names, conv, a):
        kw[n] = c(v)
    main(**kw)
