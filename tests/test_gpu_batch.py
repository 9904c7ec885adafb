"""Batched ensembles (one persistent launch) against the same jobs run alone.

Every job of a batch must give bit for bit the trajectory it gives alone
through okpz_init/okpz_sweep (itself pinned to the oracle): the same exact
width sums at every sampling time, the same final lattice and H0, for any
execution mapping of the persistent launch.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

MIXED = [  # (Lx, Ly, p, q, seed, t_max)
    (32, 32, 1.0, 0.0, 11, 9), (64, 64, 0.95, 0.05, 12, 13), (96, 96, 1.0, 0.0, 13, 7),
    (128, 64, 0.3, 0.8, 14, 10), (256, 256, 1.0, 0.0, 15, 12), (320, 192, 0.5, 0.5, 16, 6),
    (512, 512, 1.0, 0.0, 17, 5), (1056, 96, 0.95, 0.05, 18, 4), (32, 32, 0.0, 0.0, 19, 3),
    (64, 32, 1.0, 0.0, 20, 0), (2080, 64, 1.0, 1.0, 21, 5),
]
M = 0.3


@pytest.fixture(scope="module")
def okpz():
    from paper_1110_6745_amd import okpz as m

    return m


def alone(okpz, job, m, cells=0):
    Lx, Ly, p, q, seed, t_max = job
    sim = okpz.okpz_init(Lx, Ly, p, q, seed)
    sim.set_cell_borders(cells)
    out = []
    for t in okpz.sampling_times(t_max, m):
        out.append((t,) + sim.width(t))
    lat, h0 = sim.get_lattice(), sim.h0()
    sim.free()
    return out, lat, h0


def check_batch(okpz, b, jobs, m, refs):
    for r, job in enumerate(jobs):
        t, s1, s2 = b.samples(r)
        ref, lat, h0 = refs[r]
        got = list(zip(t.tolist(), s1.tolist(), s2.tolist()))
        assert got == ref, f"job {r} {job}: samples differ"
        assert np.array_equal(b.get_lattice(r), lat), f"job {r} {job}: lattice differs"
        assert b.h0(r) == h0, f"job {r} {job}: H0 differs"


def test_batch_matches_jobs_run_alone(okpz):
    refs = [alone(okpz, j, M) for j in MIXED]
    b = okpz.Batch(MIXED, M)
    b.run()
    check_batch(okpz, b, MIXED, M, refs)
    b.free()


def test_sliced_run_equals_one_launch(okpz):
    # the run in wall-clock slices (okpz_batch_start / okpz_batch_run_for):
    # launches stop taking work mid-run and the next one continues; the
    # results are those of the jobs alone, whatever the slice length
    jobs = MIXED + [(1024, 1024, 1.0, 0.0, 31, 60), (512, 256, 0.95, 0.05, 32, 80)]
    refs = [alone(okpz, j, M) for j in jobs]
    for slice_ms in (0.05, 0.5, 5.0):
        b = okpz.Batch(jobs, M)
        seen = []
        b.run(slice_ms=slice_ms, progress=seen.append)
        assert seen[-1] == len(jobs) and seen == sorted(seen)
        if slice_ms == 0.05:
            assert len(seen) > 2, "the slices did not stop the launches early"
        check_batch(okpz, b, jobs, M, refs)
        b.free()
    b = okpz.Batch(jobs, M)
    with pytest.raises(okpz.OkpzError):
        _ = okpz._bcheck(okpz._lib.okpz_batch_run_for(b._h, 1.0, None))
    b.free()


def test_batch_small_jobs_match_oracle(okpz):
    jobs = [(32, 32, 1.0, 0.0, 5, 12), (64, 96, 0.95, 0.05, 6, 8)]
    b = okpz.Batch(jobs, M)
    b.run()
    for r, (Lx, Ly, p, q, seed, t_max) in enumerate(jobs):
        lat = oracle.flat(Lx, Ly)
        H0 = oracle.run(lat, p, q, seed, 0, t_max, 0)
        assert np.array_equal(b.get_lattice(r), lat) and b.h0(r) == H0
        t, s1, s2 = b.samples(r)
        assert t[-1] == t_max and (s1[-1], s2[-1]) == oracle.width_sums(lat, H0)
    b.free()


@pytest.mark.parametrize("threads,wgs", [(256, 0), (512, 0), (1024, 5)])
def test_delayed_cell_borders_in_a_batch(okpz, threads, wgs):
    # every job of a delayed-border batch follows its lone delayed-border
    # trajectory (itself pinned to the oracle); small jobs also checked
    # against the oracle directly
    D = okpz.OKPZ_CELLS_DELAYED
    refs = [alone(okpz, j, M, D) for j in MIXED]
    b = okpz.Batch(MIXED, M)
    b.set_cell_borders(D)
    assert b.cell_borders() == D
    b.set_mapping(threads, wgs)
    b.run()
    check_batch(okpz, b, MIXED, M, refs)
    for r in (0, 3):
        Lx, Ly, p, q, seed, t_max = MIXED[r]
        lat = oracle.flat(Lx, Ly)
        H0 = oracle.run(lat, p, q, seed, 0, t_max, 0, delayed=True)
        assert np.array_equal(b.get_lattice(r), lat) and b.h0(r) == H0
    with pytest.raises(okpz.OkpzError):
        b.set_cell_borders(7)
    b.free()


@pytest.mark.parametrize("threads,wgs", [(256, 0), (512, 96), (1024, 7), (1024, 0)])
def test_mapping_does_not_change_results(okpz, threads, wgs):
    refs = [alone(okpz, j, M) for j in MIXED[:8]]
    b = okpz.Batch(MIXED[:8], M)
    b.set_mapping(threads, wgs)
    b.run()
    check_batch(okpz, b, MIXED[:8], M, refs)
    b.free()


GROWTH = [(Lx, Ly, 1.0, 0.0, seed, t) for (Lx, Ly, _, _, seed, t) in MIXED]


@pytest.mark.parametrize("cells", [0, 1])
@pytest.mark.parametrize("threads,wgs", [(256, 0), (512, 0), (1024, 0), (1024, 9)])
def test_growth_only_table(okpz, threads, wgs, cells):
    # every job p = 1, q = 0: the launch runs the growth-only kernel; the same
    # shapes as MIXED (every block size, partial bands and groups), each job
    # bit for bit its lone trajectory, for every mapping and both borders
    D = okpz.OKPZ_CELLS_DELAYED if cells else okpz.OKPZ_CELLS_DEAD
    refs = [alone(okpz, j, M, D) for j in GROWTH]
    b = okpz.Batch(GROWTH, M)
    assert b.mapping()[0] == 1024  # the default for growth-only tables
    b.set_cell_borders(D)
    b.set_mapping(threads, wgs)
    b.run()
    check_batch(okpz, b, GROWTH, M, refs)
    b.free()


def test_default_mapping_of_mixed_tables(okpz):
    b = okpz.Batch(MIXED[:4], M)
    assert b.mapping()[0] == 512
    b.free()


def test_many_tiny_jobs(okpz):
    jobs = [(32 * (1 + r % 4), 32, 1.0 if r % 2 else 0.9, 0.0 if r % 3 else 0.1, 100 + r,
             5 + r % 17) for r in range(300)]
    b = okpz.Batch(jobs, 0.5)
    b.run()
    for r in (0, 1, 2, 3, 17, 150, 299):
        ref, lat, h0 = alone(okpz, jobs[r], 0.5)
        t, s1, s2 = b.samples(r)
        assert list(zip(t.tolist(), s1.tolist(), s2.tolist())) == ref
        assert np.array_equal(b.get_lattice(r), lat) and b.h0(r) == h0
    b.free()


def test_autotune_then_run(okpz):
    jobs = MIXED[:6]
    refs = [alone(okpz, j, M) for j in jobs]
    b = okpz.Batch(jobs, M)
    threads, wgs = b.autotune(3)
    assert threads in (256, 512, 1024) and wgs > 0
    assert b.mapping() == (threads, wgs)
    b.run()
    check_batch(okpz, b, jobs, M, refs)
    # a second run repeats the first exactly
    b.run()
    check_batch(okpz, b, jobs, M, refs)
    b.free()


def test_single_large_job_equals_alone(okpz):
    # one lattice alone in a persistent launch: every sweep's 64 groups are
    # spread over the resident workgroups and handed over across XCDs
    jobs = [(2048, 2048, 0.95, 0.05, 41, 25)]
    refs = [alone(okpz, j, 0.2) for j in jobs]
    b = okpz.Batch(jobs, 0.2)
    b.run()
    check_batch(okpz, b, jobs, 0.2, refs)
    b.free()


def test_large_and_small_lattices_in_one_launch(okpz):
    jobs = [(4096, 4096, 1.0, 0.0, 31, 6), (2048, 2048, 0.95, 0.05, 32, 8),
            (8192, 256, 1.0, 0.0, 33, 5), (64, 64, 1.0, 0.0, 34, 40), (32, 96, 0.5, 0.5, 35, 30)]
    refs = [alone(okpz, j, 0.5) for j in jobs]
    b = okpz.Batch(jobs, 0.5)
    b.run()
    check_batch(okpz, b, jobs, 0.5, refs)
    b.free()


def test_steady_state_statistics_match_oracle(okpz):
    # cumulants (Eq. (cumulants)) and Psi_L of the batch's samples against
    # the oracle's exact statistics of its own runs of the same realizations
    from oracle import stats

    m, t_max, t_from, R = 0.05, 120, 40, 6
    groups = [(32, 1.0, 0.0, 100), (64, 0.95, 0.05, 200)]
    jobs = [(L, L, p, q, s0 + r, t_max) for (L, p, q, s0) in groups for r in range(R)]
    b = okpz.Batch(jobs, m)
    b.run()
    times = [t for t in oracle.sampling_times(t_max, m) if t >= t_from]
    for L, p, q, s0 in groups:
        ens = oracle.ensemble(L, L, p, q, s0, R, t_max)  # S1, S2 after MCS 1..t_max
        vals = [stats.w2_exact(int(ens[r, t - 1, 0]), int(ens[r, t - 1, 1]), L * L)
                for r in range(R) for t in times]
        nu_x = [float(v) for v in stats.moments(vals)]
        k_x = [float(v) for v in stats.cumulants(vals)]
        n, nu, kappa = b.w2_cumulants(L, L, t_from)
        assert n == len(vals)
        for i in range(4):
            assert nu[i] == pytest.approx(nu_x[i], rel=1e-12)
            scale = abs(k_x[1]) ** ((i + 1) / 2)
            assert abs(kappa[i] - k_x[i]) <= 1e-9 * (abs(k_x[i]) + scale)
        x_hi, nb = 3.0, 24
        ps, cnt = b.psi(L, L, t_from, x_hi, nb)
        ps_x = stats.psi(vals, x_hi, nb)
        assert cnt == len(vals)
        # at most one sample on a bin edge may fall on the other side
        assert np.abs(ps - np.array(ps_x)).sum() <= 2.0 / (cnt * x_hi / nb) + 1e-12
    b.free()
