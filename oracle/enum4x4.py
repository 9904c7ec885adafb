"""Exact master-equation evolution of the octahedron model on a 4x4 torus.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

This module is independent of the C oracle: it works on height functions
(Sec. I: heights are reconstructed from the slopes) instead of slope bits,
enumerates every valid periodic configuration, and builds the exact
transition matrices of

* the random-sequential chain: one attempt picks a uniform site; a local
  height minimum is raised by 2 with probability p, a local maximum lowered
  by 2 with probability q (Eq. (1)); one MCS = N attempts;
* the seeded tiled chain on a 4x4 lattice (one 4x4 device-level block,
  one 4x4 thread cell, Sec. II): per MCS a uniform block shift, then C^2 = 16
  steps, each with a uniform cell origin and one site drawn among the cell's
  (C-1)^2 = 9 active sites with the exact probabilities of the 16-bit draw
  ``floor(h16 * 9 / 2^16)``; sites on the block's dead border do nothing;
* the same chain with delayed cell borders (Sec. II): the site is drawn among
  all 16 sites of the cell (``floor(h16 * 16 / 2^16)``, exactly uniform);
  with a single cell per block the bulk / edge / corner order of a step has
  nothing to order, so only the draw and the block border matter.

Both chains start from the flat zig-zag state (Sec. III) and give the exact
law of W^2(t) (Eq. (Wdef)), against which Monte Carlo histograms of the C
oracle are tested.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
import itertools

import numpy as np

L = 4
N = L * L


def _heights_from_state(state: tuple) -> np.ndarray:
    """Heights (h(0,0) = 0) of a state given as (bx bits, by bits) tuples."""
    bx = np.array(state[:N], dtype=np.int64).reshape(L, L)
    by = np.array(state[N:], dtype=np.int64).reshape(L, L)
    sx, sy = 2 * bx - 1, 2 * by - 1
    h = np.zeros((L, L), dtype=np.int64)
    for y in range(L):
        if y > 0:
            h[y, 0] = h[y - 1, 0] + sy[y - 1, 0]
        for x in range(1, L):
            h[y, x] = h[y, x - 1] + sx[y, x - 1]
    return h


def _state_from_heights(h: np.ndarray) -> tuple:
    sx = np.roll(h, -1, axis=1) - h
    sy = np.roll(h, -1, axis=0) - h
    assert np.all(np.abs(sx) == 1) and np.all(np.abs(sy) == 1)
    bx = (sx > 0).astype(np.int64).ravel()
    by = (sy > 0).astype(np.int64).ravel()
    return tuple(int(v) for v in bx) + tuple(int(v) for v in by)


@lru_cache(maxsize=None)
def states() -> tuple:
    """All valid periodic 4x4 configurations, found by breadth-first search
    over single-site moves from the flat state, then cross-checked by a direct
    enumeration of slope fields (see ``states_by_slopes``)."""
    h0 = np.add.outer(np.arange(L), np.arange(L)) % 2  # flat: h = (x+y) mod 2
    start = _state_from_heights(h0)
    seen = {start}
    frontier = [start]
    while frontier:
        nxt = []
        for st in frontier:
            h = _heights_from_state(st)
            for y in range(L):
                for x in range(L):
                    k = _kind(h, x, y)
                    if k == 0:
                        continue
                    h2 = h.copy()
                    h2[y, x] += 2 * k
                    s2 = _state_from_heights(h2)
                    if s2 not in seen:
                        seen.add(s2)
                        nxt.append(s2)
        frontier = nxt
    return tuple(sorted(seen))


def states_by_slopes() -> tuple:
    """Direct enumeration: every slope field with zero row sums of sigma_x,
    zero column sums of sigma_y and closed plaquettes (curl-free)."""
    rows = [r for r in itertools.product((0, 1), repeat=L) if sum(r) == L // 2]
    out = []
    for bxr in itertools.product(rows, repeat=L):
        bx = np.array(bxr)  # bx[y][x]
        for byc in itertools.product(rows, repeat=L):
            by = np.array(byc).T  # column sums zero: by[y][x] = byc[x][y]
            sx, sy = 2 * bx - 1, 2 * by - 1
            curl = sx + np.roll(sy, -1, axis=1) - np.roll(sx, -1, axis=0) - sy
            if np.all(curl == 0):
                out.append(tuple(int(v) for v in bx.ravel()) + tuple(int(v) for v in by.ravel()))
    return tuple(sorted(out))


def _kind(h: np.ndarray, x: int, y: int) -> int:
    """+1 local minimum, -1 local maximum, 0 otherwise (Eq. (1))."""
    c = h[y, x]
    nb = (h[y, (x + 1) % L], h[y, (x - 1) % L], h[(y + 1) % L, x], h[(y - 1) % L, x])
    if all(v == c + 1 for v in nb):
        return +1
    if all(v == c - 1 for v in nb):
        return -1
    return 0


@lru_cache(maxsize=None)
def index() -> dict:
    return {s: i for i, s in enumerate(states())}


def w2_exact(state: tuple) -> Fraction:
    h = _heights_from_state(state)
    s1 = int(h.sum())
    s2 = int((h * h).sum())
    return Fraction(N * s2 - s1 * s1, N * N)


@lru_cache(maxsize=None)
def w2_values() -> np.ndarray:
    return np.array([float(w2_exact(s)) for s in states()])


def flat_index() -> int:
    h0 = np.add.outer(np.arange(L), np.arange(L)) % 2
    return index()[_state_from_heights(h0)]


@lru_cache(maxsize=None)
def _moves() -> tuple:
    """For every site: (target index, kind) per state (kind 0: no move)."""
    idx = index()
    S = len(idx)
    tgt = np.zeros((N, S), dtype=np.int64)
    kind = np.zeros((N, S), dtype=np.int64)
    for i, st in enumerate(states()):
        h = _heights_from_state(st)
        for y in range(L):
            for x in range(L):
                k = _kind(h, x, y)
                site = y * L + x
                kind[site, i] = k
                if k == 0:
                    tgt[site, i] = i
                else:
                    h2 = h.copy()
                    h2[y, x] += 2 * k
                    tgt[site, i] = idx[_state_from_heights(h2)]
    return tgt, kind


def site_matrix(x: int, y: int, p: float, q: float) -> np.ndarray:
    """Row-stochastic matrix of one update attempt at site (x, y)."""
    tgt, kind = _moves()
    S = tgt.shape[1]
    site = y * L + x
    pr = np.where(kind[site] > 0, p, np.where(kind[site] < 0, q, 0.0))
    M = np.zeros((S, S))
    rows = np.arange(S)
    np.add.at(M, (rows, tgt[site]), pr)
    np.add.at(M, (rows, rows), 1.0 - pr)
    return M


def rsu_mcs_matrix(p: float, q: float) -> np.ndarray:
    """One MCS of the random-sequential chain: (mean single attempt)^N."""
    M1 = sum(site_matrix(x, y, p, q) for y in range(L) for x in range(L)) / N
    return np.linalg.matrix_power(M1, N)


def draw_probabilities(C: int) -> np.ndarray:
    """Exact law of the active-site index floor(h16*(C-1)^2/2^16), h16 uniform."""
    A = (C - 1) * (C - 1)
    h = np.arange(1 << 16, dtype=np.int64)
    return np.bincount((h * A) >> 16, minlength=A) / float(1 << 16)


@lru_cache(maxsize=None)
def translation(dx: int, dy: int) -> np.ndarray:
    """perm[i] = index of the state whose slopes at (x, y) are those of
    state i at (x + dx, y + dy)."""
    idx = index()
    perm = np.empty(len(idx), dtype=np.int64)
    for i, st in enumerate(states()):
        bx = np.array(st[:N]).reshape(L, L)
        by = np.array(st[N:]).reshape(L, L)
        bx2 = np.roll(bx, (-dy, -dx), axis=(0, 1))
        by2 = np.roll(by, (-dy, -dx), axis=(0, 1))
        perm[i] = idx[tuple(int(v) for v in bx2.ravel()) + tuple(int(v) for v in by2.ravel())]
    return perm


def tiled_site_weights(C: int = 4, delayed: bool = False) -> np.ndarray:
    """Probability that a step attempts block-local site (u, v), shape (L, L);
    entries with u = 0 or v = 0 are dead-border no-ops."""
    if delayed:
        h = np.arange(1 << 16, dtype=np.int64)
        P = np.bincount((h * C * C) >> 16, minlength=C * C) / float(1 << 16)
    else:
        P = draw_probabilities(C)
    w = np.zeros((L, L))
    for oy in range(C):
        for ox in range(C):
            for i in range(len(P)):
                if delayed:
                    a, b = i % C, i // C
                else:
                    a, b = 1 + i % (C - 1), 1 + i // (C - 1)
                w[(oy + b) % L, (ox + a) % L] += P[i] / (C * C)
    return w


def tiled_step_matrix(sx: int, sy: int, p: float, q: float, delayed: bool = False) -> np.ndarray:
    """One step of the tiled chain under block shift (sx, sy), built directly."""
    w = tiled_site_weights(delayed=delayed)
    S = len(states())
    step = np.zeros((S, S))
    for v in range(L):
        for u in range(L):
            if u == 0 or v == 0:
                step += w[v, u] * np.eye(S)
            else:
                step += w[v, u] * site_matrix((sx + u) % L, (sy + v) % L, p, q)
    return step


def tiled_mcs_matrix(p: float, q: float, delayed: bool = False) -> np.ndarray:
    """One MCS of the tiled chain on the 4x4 torus (B = C = 4): the average
    over the L*L block shifts of (step matrix)^(C*C).  The step under shift d
    is the shift-0 step conjugated by the translation by d."""
    C = 4
    P16 = np.linalg.matrix_power(tiled_step_matrix(0, 0, p, q, delayed), C * C)
    total = np.zeros_like(P16)
    for sy in range(L):
        for sx in range(L):
            perm = translation(sx, sy)
            total += P16[np.ix_(perm, perm)]
    return total / (L * L)


def evolve(M: np.ndarray, t_list) -> dict:
    """Law of the state at each time in ``t_list`` (MCS), from the flat state."""
    S = M.shape[0]
    pi = np.zeros(S)
    pi[flat_index()] = 1.0
    out = {}
    t = 0
    for target in sorted(t_list):
        while t < target:
            pi = pi @ M
            t += 1
        out[target] = pi.copy()
    return out


def w2_law(pi: np.ndarray) -> dict:
    """Distribution of W^2 (keyed by the exact value) for a state law pi."""
    law = {}
    for s, pr in zip(states(), pi):
        w = w2_exact(s)
        law[w] = law.get(w, 0.0) + pr
    return law


def mean_w2(pi: np.ndarray) -> float:
    return float(pi @ w2_values())
