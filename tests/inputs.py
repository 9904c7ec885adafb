"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds sizes, seeds and parameter lists only.  Rough start states are produced
by the oracle (``oracle.rsu_run``), never by the HIP path.  Every workload
starts from the flat zig-zag state and is driven by a seed, as in the paper's
runs (Sec. III); there is no dataset.
"""
import numpy as np

# (p, q) pairs: pure growth, the paper-style asymmetric pair, symmetric, and
# degenerate endpoints.
PQ_GROWTH = (1.0, 0.0)
PQ_ASYM = (0.95, 0.05)
PQ_SYM = (0.5, 0.5)
PQ_LIST = [PQ_GROWTH, PQ_ASYM, PQ_SYM, (0.3, 0.8), (0.0, 1.0), (0.0, 0.0)]

# lattice shapes: square powers of two, ragged block sizes (power-of-two
# divisor below 256), rectangles
SHAPES_SMALL = [(4, 4), (8, 8), (12, 20), (32, 32), (96, 64), (64, 160)]
SHAPES_GPU = [(32, 32), (64, 32), (96, 96), (256, 256), (320, 192), (512, 1024), (1056, 96),
              (2080, 64), (128, 640)]


def rough_state(Lx, Ly, seed, mcs=3, p=0.7, q=0.4):
    """A valid non-flat slope field: the flat state evolved by the oracle's
    random-sequential reference for a few MCS.  Returns (lattice, H0)."""
    import oracle

    lat = oracle.flat(Lx, Ly)
    H0 = oracle.rsu_run(lat, p, q, seed, 0, mcs, 0)
    return lat, H0


def random_bytes(n, seed):
    return np.random.default_rng(seed).integers(0, 256, size=n, dtype=np.uint8)
