"""Benchmark of the octahedron-model hot path on one MI355X.

Workload: 2^17 x 2^17 periodic lattice (1.7e10 sites, 4.3 GB packed), flat
zig-zag start, p = 1, q = 0, seed 1, with the exact width measured at the
paper's sampling times t_{i+1} = (t_i + 10) e^m, m = 0.01 (Sec. III).  One
step is one MCS: a full sweep (every block staged in LDS, 64 in-LDS steps,
aligned store) plus the width whenever a sampling time falls on it.  W
untimed warmup sweeps run first; then exactly K steps are timed.

Prints one JSON line: whole-job site updates/s, the sweep kernel's HBM
roofline fraction (algorithmic 0.5 B per site update over the kernel's mean
launch time, measured with HIP events on the simulation's stream), and the
oracle timed on the host cores on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "site updates/s (+% HBM roofline) at L=2^17; realizations/s batched vs plain"


def sampling_times(tmax, m=0.01):
    """ceil of t_{i+1} = (t_i + 10) e^m, t_0 = 0 (Sec. III), up to tmax."""
    out, t = [], 0.0
    while True:
        t = (t + 10.0) * math.exp(m)
        if t > tmax:
            return sorted(set(out))
        out.append(int(math.ceil(t)))


def cpu_baseline(budget_s=12.0):
    """The oracle, untuned, on the host cores: MCS of a 4096^2 flat lattice,
    p = 1, q = 0, seed 1 -- 256 blocks of the same 256 x 256 geometry and
    schedule as the 2^17 workload, so the per-site work is identical."""
    import oracle

    L = 4096
    lat = oracle.flat(L, L)
    threads = oracle.num_threads()
    H0, s, t0 = 0, 0, time.perf_counter()
    while True:
        H0 = oracle.sweep(lat, 1.0, 0.0, 1, s, H0)
        s += 1
        el = time.perf_counter() - t0
        if el >= budget_s or s >= 400:
            break
    return {"value": L * L * s / el, "unit": "site updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{s} MCS of a 4096x4096 flat lattice (p=1, q=0, seed 1; 256 blocks of the "
                      f"2^17 workload's 256x256 geometry), {el:.1f} s, OpenMP over blocks"}


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--L", type=int, default=1 << 17)
    ap.add_argument("--threads", type=int, default=1024, help="sweep workgroup size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib", action="store_true", help="run a 1 GiB copy first (counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); independent "
              "realizations shard trivially and one lattice is not split across GPUs here",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1110_6745_amd import okpz

    torch.cuda.set_device(0)
    if args.calib:
        copy_calibration()
    L = args.L
    p, q, seed = 1.0, 0.0, 1
    N = L * L
    nbytes = okpz.okpz_required_bytes(L, L)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sim = okpz.okpz_init_on(L, L, p, q, seed, buf.data_ptr(), nbytes, stream.cuda_stream)
    sim.set_threads(args.threads)

    sim.sweep(args.warmup)
    torch.cuda.synchronize()
    t_lo, t_hi = args.warmup, args.warmup + args.steps
    samples = [t for t in sampling_times(t_hi) if t_lo < t <= t_hi]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    widths = []

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        sim.sweep(1)
        ev[i][1].record(stream)
        if (t_lo + i + 1) in samples:
            widths.append((t_lo + i + 1,) + sim.width())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    sweep_ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    value = N * args.steps / elapsed
    achieved_gbs = 0.5 * N / (sweep_ms * 1e-3) / 1e9
    w2 = [(t, (N * s2 - s1 * s1) / (N * N)) for t, s1, s2 in widths]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"octahedron model {L}x{L} periodic, flat init, p=1 q=0, seed 1, "
                               f"MCS {t_lo}..{t_hi}, exact W^2 at t_(i+1)=(t_i+10)e^0.01",
                   "Lx": L, "Ly": L, "p": p, "q": q, "seed": seed,
                   "width_samples": len(widths), "threads_per_workgroup": args.threads},
        "sweep_kernel_ms": sweep_ms,
        "sweep_site_updates_per_s": N / (sweep_ms * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None},
        "w2_last": w2[-1] if w2 else None,
    }
    sim.free()
    del buf
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
