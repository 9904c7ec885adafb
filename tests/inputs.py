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


# ---------------------------------------------------------------------------
# Large synthetic surfaces for the width at full size.  A height function is
# built from closed +-1 walks, which gives a valid periodic slope field by
# construction (no dynamics involved):
#   separable: h(x,y) = H0 + A(x) + B(y), so sigma_x(x,y) = a(x), sigma_y = b(y);
#   diagonal (Lx = Ly = L): h(x,y) = H0 + A((x + y) mod L), so both slopes of
#     site (x,y) are a((x + y) mod L) and every row is a rotated copy of one
#     walk.
# A walk is a seeded shuffle of L/2 up and L/2 down steps (bits 1/0).
# ---------------------------------------------------------------------------
def balanced_bits(L, seed):
    bits = np.zeros(L, dtype=np.uint8)
    bits[: L // 2] = 1
    np.random.default_rng(seed).shuffle(bits)
    return bits


def separable_rows(a, b, y0, n):
    """Canonical bytes of rows y0 .. y0+n-1 of the separable surface."""
    return np.ascontiguousarray(a[None, :] | (b[y0:y0 + n, None] << 1))


def diagonal_rows(a, y0, n):
    """Canonical bytes of rows y0 .. y0+n-1 of the diagonal surface."""
    L = a.size
    a3 = np.concatenate([a, a]) * np.uint8(3)
    view = np.lib.stride_tricks.as_strided(a3[y0 % L:], shape=(n, L), strides=(1, 1))
    return np.ascontiguousarray(view)


def _pack_bits(bits):
    """Bit j of word w is column 32 w + j."""
    return np.packbits(bits, bitorder="little").view("<u4")


def checkpoint_of(kind, a, b, H0, seed=1, t=0):
    """An okpz checkpoint (okpz_save layout: 80-byte header, then the sigma_x
    and sigma_y bit planes [Ly][Lx/32] of uint32) holding the separable or
    diagonal surface, as one uint8 array, with columns stored unrotated."""
    import struct

    L = a.size
    Ly = b.size if kind == "separable" else L
    W = L // 32
    buf = np.empty(80 + 2 * Ly * W * 4, dtype=np.uint8)
    buf[:80] = np.frombuffer(struct.pack("<8sIIqqddQqqii", b"OKPZCKP1", 1, 0, L, Ly, 1.0, 0.0,
                                         seed, t, H0, 0, 2), dtype=np.uint8)
    planes = buf[80:].view("<u4").reshape(2, Ly, W)
    if kind == "separable":
        planes[0] = _pack_bits(a)[None, :]
        planes[1] = np.where(b[:, None] == 1, np.uint32(0xFFFFFFFF), np.uint32(0))
    else:
        # row y holds a rotated left by y sites: rotations by whole words are
        # word rotations of one of the 32 bit-shifted copies
        a2 = np.concatenate([a, a])
        for j in range(32):
            w = _pack_bits(a2[j:j + L])
            w2 = np.concatenate([w, w])
            rows = np.lib.stride_tricks.as_strided(w2, shape=(W, W), strides=(4, 4))
            planes[0, j::32] = rows[: len(range(j, Ly, 32))]
        planes[1] = planes[0]
    return buf
