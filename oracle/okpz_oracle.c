/*
 * okpz oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the hot path
 * computes, for the octahedron model of Kelling & Odor, "Extremely large
 * scale simulation of a KPZ model using graphics cards" (arXiv:1110.6745).
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or constant generator
 * with the HIP library; it implements its own Philox4x32-10.
 *
 * Lattice representation (oracle only): one byte per site, row-major
 * lat[y*Lx + x]; bit 0 = bx = [sigma_x(x,y) = +1], bit 1 = by =
 * [sigma_y(x,y) = +1], with sigma_x(x,y) = h(x+1,y) - h(x,y) and
 * sigma_y(x,y) = h(x,y+1) - h(x,y) (forward differences stored at the site;
 * Sec. II: two bits per site, two slopes stored off-site, Fig. 1 caption).
 *
 * Parity status of each function is stated at the function.  The seeded
 * tiled schedule (or_block_sweep / or_sweep) has no worked example in the
 * paper: it is pinned by the model invariants, the mirror symmetry, the
 * flat-state closed form and the exact 4x4 master-equation enumeration
 * (tests), not by printed values.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11.  Counter-based: out = bijection_key(counter).    */
/* The paper itself used per-thread 32-bit LCRNGs (Sec. II); the counter-    */
/* based generator replaces them so a trajectory is a pure function of seed. */
/* ------------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u; /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u; /* Weyl key increments */
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream tags (fourth counter word).  Each random decision of the dynamics
 * has its own counter, so no decision depends on execution order. */
enum { TAG_SITE = 0, TAG_ORIGIN = 1, TAG_SHIFT = 2, TAG_RSU = 3, TAG_ACCEPT = 4 };

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    or_philox(ctr, key, out);
}

/* Uniform integer in [0, n) from a 32-bit word: floor(r * n / 2^32). */
static uint32_t uniform_below(uint32_t r, uint32_t n)
{
    return (uint32_t)(((uint64_t)r * (uint64_t)n) >> 32);
}

/* Acceptance threshold for a probability (Eq. (1): attachment with p,
 * detachment with q).  A move is accepted iff the 32-bit draw is < T. */
uint64_t or_threshold(double prob)
{
    if (!(prob > 0.0)) return 0;               /* also maps NaN to 0 */
    if (prob >= 1.0) return (uint64_t)1 << 32;
    double t = ldexp(prob, 32);
    long long r = llround(t);
    if (r < 0) r = 0;
    if (r > (1LL << 32)) r = 1LL << 32;
    return (uint64_t)r;
}

/* Geometry of the two-level dead-border decomposition (Sec. II):
 * block side = largest power of two dividing L, at most 256 (the paper's
 * block-border ratio of about 1/128 corresponds to 256-site blocks); thread
 * cell side = min(8, Bx, By) (the paper's 8x8 thread cell). */
static int64_t pow2_divisor_capped(int64_t L, int64_t cap)
{
    int64_t b = 1;
    while (b < cap && (L % (b * 2)) == 0) b *= 2;
    return b;
}

int or_geometry(int64_t Lx, int64_t Ly, int32_t *Bx, int32_t *By, int32_t *C)
{
    if (Lx < 4 || Ly < 4 || (Lx % 4) != 0 || (Ly % 4) != 0) return -1;
    int64_t bx = pow2_divisor_capped(Lx, 256), by = pow2_divisor_capped(Ly, 256);
    int64_t c = 8;
    if (bx < c) c = bx;
    if (by < c) c = by;
    *Bx = (int32_t)bx; *By = (int32_t)by; *C = (int32_t)c;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Flat initial state (Sec. III: half-filled zig-zag surface, W^2 = 1/4).    */
/* h(x,y) = (x+y) mod 2, so bx = by = [x+y even] and h(0,0) = 0.             */
/* ------------------------------------------------------------------------ */
void or_flat(uint8_t *lat, int64_t Lx, int64_t Ly)
{
    for (int64_t y = 0; y < Ly; ++y)
        for (int64_t x = 0; x < Lx; ++x) {
            uint8_t up = ((x + y) % 2 == 0) ? 1 : 0;
            lat[y * Lx + x] = (uint8_t)(up | (up << 1));
        }
}

/* ------------------------------------------------------------------------ */
/* Generalized Kawasaki rule at one site (Eq. (1)).                           */
/* The four slopes meeting at (x,y) are A = sigma_x(x-1,y), B = sigma_x(x,y), */
/* Cc = sigma_y(x,y-1), D = sigma_y(x,y).  Matrix rows are the x and y        */
/* directions, columns the bond behind / ahead of the site:                   */
/*   (A B; Cc D) = (-1 +1; -1 +1) is a local minimum -> flipped to the        */
/*   maximum (+1 -1; +1 -1) with probability p (attachment, h += 2), and the  */
/*   reverse with probability q (detachment, h -= 2).                         */
/* Returns +1 if the site is a local minimum, -1 if a local maximum, else 0.  */
/* ------------------------------------------------------------------------ */
static int site_kind(int A, int B, int Cc, int D)
{
    if (A == -1 && B == +1 && Cc == -1 && D == +1) return +1;
    if (A == +1 && B == -1 && Cc == +1 && D == -1) return -1;
    return 0;
}

static int bit_to_slope(int bit) { return bit ? +1 : -1; }

/* ------------------------------------------------------------------------ */
/* One Monte Carlo step of one device-level block (Sec. II).                 */
/*                                                                          */
/* blk: Bx*By bytes, the block's sites cut out of the periodic lattice,      */
/*      blk[v*Bx + u] for block-local (u, v).                                */
/* The block updates sites with u >= 1 and v >= 1 only: u = 0 and v = 0 are   */
/* its dead borders (two edges only, since each site stores the two slopes   */
/* towards +x and +y), so every bond an update touches is stored inside the  */
/* block and no other block touches it.                                      */
/*                                                                          */
/* Thread-cell level: C*C steps; at step k the cell origin (ox, oy) is drawn */
/* afresh (the paper redraws it at every attempt, 64 times per MCS); cell c   */
/* covers block-local ((ox + cx*C + a) mod Bx, (oy + cy*C + b) mod By) for    */
/* a, b in [0, C); a = 0 or b = 0 is the cell's dead border; each cell draws  */
/* one site among its (C-1)^2 active sites per step.  A site on the block's   */
/* dead border does nothing.  Two sites attempted in one step are never      */
/* nearest neighbours, so their bond sets are disjoint and the order of the  */
/* attempts inside a step does not matter.                                   */
/*                                                                          */
/* Random numbers (counter = (c0, c1, c2, c3), key = seed):                  */
/*   cell origin of steps 2m, 2m+1:  (s, id, m, ORIGIN) -> words 0,1 / 2,3    */
/*   site of cell c at step k:       (s, id, (k/8)<<16 | c, SITE), 16-bit     */
/*                                   half (k mod 8) of the 128-bit output     */
/*   acceptance of cell c, step k:   (s, id, (k/4)<<16 | c, ACCEPT), word     */
/*                                   (k mod 4)                                */
/*                                                                          */
/* site00_u/v: block-local position of lattice site (0,0), or -1; *dh00      */
/* accumulates its height change (the absolute height reference).            */
/* touched: NULL, or 2*Bx*By bytes of scratch for the bond-conflict check.   */
/*                                                                          */
/* delayed != 0 selects the delayed thread-cell borders of Sec. II instead   */
/* of dead ones: each cell draws one of all C*C sites, i = floor(h16 C^2 /   */
/* 2^16), a = i mod C, b = i div C; at every step the attempts on cell-bulk  */
/* sites (a, b >= 1) come first, then those on the cell's edges (exactly one */
/* of a, b zero), then those on its corner (a = b = 0).  Attempts of one     */
/* phase are never nearest neighbours, so each phase is order independent;   */
/* the conflict check covers one phase at a time.  Needs C >= 2.            */
/* Returns 0, or -1 if a bond was touched twice within one step (phase).    */
/* ------------------------------------------------------------------------ */
int or_block_sweep(uint8_t *blk, int32_t Bx, int32_t By, int32_t C, uint64_t seed,
                   uint32_t s, uint32_t id, uint64_t Tp, uint64_t Tq,
                   int32_t site00_u, int32_t site00_v, int64_t *dh00,
                   int64_t *n_att, int64_t *n_det, uint8_t *touched, int delayed)
{
    const int32_t ncx = Bx / C, ncy = By / C, ncell = ncx * ncy;
    const uint32_t nact = delayed ? (uint32_t)(C * C) : (uint32_t)((C - 1) * (C - 1));
    const int nphase = delayed ? 3 : 1;
    int32_t su[1024], sv[1024], sph[1024];
    if (ncell > 1024 || (delayed && C < 2)) return -2;
    for (int32_t k = 0; k < C * C; ++k) {
        uint32_t r[4];
        draw(seed, s, id, (uint32_t)(k / 2), TAG_ORIGIN, r);
        int32_t ox = (int32_t)uniform_below((k % 2 == 0) ? r[0] : r[2], (uint32_t)C);
        int32_t oy = (int32_t)uniform_below((k % 2 == 0) ? r[1] : r[3], (uint32_t)C);

        /* every cell's site of this step */
        for (int32_t c = 0; c < ncell; ++c) {
            int32_t cx = c % ncx, cy = c / ncx;
            draw(seed, s, id, ((uint32_t)(k / 8) << 16) | (uint32_t)c, TAG_SITE, r);
            int32_t e = k % 8;
            uint32_t h16 = (r[e / 2] >> (16 * (e % 2))) & 0xffffu;
            uint32_t idx = (uint32_t)(((uint64_t)h16 * nact) >> 16);
            int32_t a, b;
            if (delayed) {
                a = (int32_t)(idx % (uint32_t)C);
                b = (int32_t)(idx / (uint32_t)C);
            } else {
                a = 1 + (int32_t)(idx % (uint32_t)(C - 1));
                b = 1 + (int32_t)(idx / (uint32_t)(C - 1));
            }
            su[c] = (ox + cx * C + a) % Bx;
            sv[c] = (oy + cy * C + b) % By;
            sph[c] = (a == 0) + (b == 0); /* 0 bulk, 1 edge, 2 corner */
        }

        for (int ph = 0; ph < nphase; ++ph) {
            if (touched) memset(touched, 0, (size_t)2 * Bx * By);
            for (int32_t c = 0; c < ncell; ++c) {
                if (delayed && sph[c] != ph) continue;
                int32_t u = su[c], v = sv[c];
                if (u == 0 || v == 0) continue; /* block-border site: no-op */

                if (touched) {
                    /* bonds: x-bond stored at (u-1,v) and (u,v), y-bond at (u,v-1) and (u,v) */
                    size_t ia = (size_t)2 * (v * Bx + (u - 1)) + 0;
                    size_t ib = (size_t)2 * (v * Bx + u) + 0;
                    size_t ic = (size_t)2 * ((v - 1) * Bx + u) + 1;
                    size_t id_ = (size_t)2 * (v * Bx + u) + 1;
                    if (touched[ia] || touched[ib] || touched[ic] || touched[id_]) return -1;
                    touched[ia] = touched[ib] = touched[ic] = touched[id_] = 1;
                }

                uint8_t *sl = &blk[v * Bx + (u - 1)];
                uint8_t *sc = &blk[v * Bx + u];
                uint8_t *sd = &blk[(v - 1) * Bx + u];
                int A = bit_to_slope(*sl & 1), B = bit_to_slope(*sc & 1);
                int Cc = bit_to_slope((*sd >> 1) & 1), D = bit_to_slope((*sc >> 1) & 1);
                int kind = site_kind(A, B, Cc, D);
                if (kind == 0) continue;

                draw(seed, s, id, ((uint32_t)(k / 4) << 16) | (uint32_t)c, TAG_ACCEPT, r);
                uint64_t racc = r[k % 4];
                int accept = (kind > 0) ? (racc < Tp) : (racc < Tq);
                if (!accept) continue;

                /* flip the four slopes: minimum <-> maximum */
                *sl ^= 1; *sc ^= 1; *sd ^= 2; *sc ^= 2;
                if (kind > 0) { if (n_att) (*n_att)++; } else { if (n_det) (*n_det)++; }
                if (u == site00_u && v == site00_v && dh00) *dh00 += (kind > 0) ? 2 : -2;
            }
        }
    }
    return 0;
}

/* Block shift of sweep s: (sx, sy) uniform in [0,Bx) x [0,By) (Sec. II: the
 * origin of the device-level decomposition is moved at every MCS; the shift
 * granularity here is one site). */
void or_block_shift(uint64_t seed, uint32_t s, int32_t Bx, int32_t By,
                    int32_t *sx, int32_t *sy)
{
    uint32_t r[4];
    draw(seed, s, 0, 0, TAG_SHIFT, r);
    *sx = (int32_t)uniform_below(r[0], (uint32_t)Bx);
    *sy = (int32_t)uniform_below(r[1], (uint32_t)By);
}

/* ------------------------------------------------------------------------ */
/* One MCS of the tiled dynamics over the whole periodic lattice: the block  */
/* (i, j) covers sites ((sx + i*Bx + u) mod Lx, (sy + j*By + v) mod Ly),     */
/* block id j*(Lx/Bx) + i.  Blocks are independent within a sweep (Sec. II,  */
/* "not communicating blocks"), so they may be processed in any order.       */
/* Returns 0, -1 on a bond conflict, -2 on bad arguments.                    */
/* ------------------------------------------------------------------------ */
int or_sweep(uint8_t *lat, int64_t Lx, int64_t Ly, uint64_t Tp, uint64_t Tq,
             uint64_t seed, uint32_t s, int64_t *H0, int64_t *n_att, int64_t *n_det,
             int check, int delayed)
{
    int32_t Bx, By, C;
    if (or_geometry(Lx, Ly, &Bx, &By, &C) != 0) return -2;
    if (delayed && C < 2) return -2;
    int32_t sx, sy;
    or_block_shift(seed, s, Bx, By, &sx, &sy);
    const int64_t nbx = Lx / Bx, nby = Ly / By, nblk = nbx * nby;
    int64_t att = 0, det = 0, dh = 0;
    int bad = 0;

#pragma omp parallel for schedule(dynamic, 16) reduction(+ : att, det, dh) reduction(| : bad) if (nblk >= 4)
    for (int64_t bid = 0; bid < nblk; ++bid) {
        int64_t i = bid % nbx, j = bid / nbx;
        int64_t x0 = sx + i * Bx, y0 = sy + j * By;
        uint8_t *blk = (uint8_t *)malloc((size_t)Bx * By);
        uint8_t *touched = check ? (uint8_t *)malloc((size_t)2 * Bx * By) : NULL;
        for (int32_t v = 0; v < By; ++v)
            for (int32_t u = 0; u < Bx; ++u)
                blk[v * Bx + u] = lat[((y0 + v) % Ly) * Lx + ((x0 + u) % Lx)];
        /* block-local position of lattice site (0,0) */
        int64_t u00 = ((0 - x0) % Lx + Lx) % Lx, v00 = ((0 - y0) % Ly + Ly) % Ly;
        int32_t su = (u00 < Bx && v00 < By) ? (int32_t)u00 : -1;
        int32_t sv = (u00 < Bx && v00 < By) ? (int32_t)v00 : -1;
        int64_t a = 0, d = 0, h = 0;
        if (or_block_sweep(blk, Bx, By, C, seed, s, (uint32_t)bid, Tp, Tq, su, sv, &h,
                           &a, &d, touched, delayed) != 0)
            bad = 1;
        for (int32_t v = 0; v < By; ++v)
            for (int32_t u = 0; u < Bx; ++u)
                lat[((y0 + v) % Ly) * Lx + ((x0 + u) % Lx)] = blk[v * Bx + u];
        att += a; det += d; dh += h;
        free(blk);
        free(touched);
    }
    if (H0) *H0 += dh;
    if (n_att) *n_att += att;
    if (n_det) *n_det += det;
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Textbook random-sequential update (statistical reference): one MCS of sweep   */
/* index t is N = Lx*Ly attempts ("one overall update", Sec. II); attempt n  */
/* picks a uniform site and applies Eq. (1).  Attempt a = t*N + n uses       */
/* counter (a mod 2^32, a / 2^32, 0, RSU): x from word 0, y from word 1,     */
/* acceptance from word 2.                                                   */
/* ------------------------------------------------------------------------ */
void or_rsu_sweep(uint8_t *lat, int64_t Lx, int64_t Ly, uint64_t Tp, uint64_t Tq,
                  uint64_t seed, uint64_t t, int64_t *H0, int64_t *n_att, int64_t *n_det)
{
    const uint64_t N = (uint64_t)Lx * (uint64_t)Ly;
    for (uint64_t n = 0; n < N; ++n) {
        uint64_t a = t * N + n;
        uint32_t r[4];
        draw(seed, (uint32_t)(a & 0xffffffffu), (uint32_t)(a >> 32), 0, TAG_RSU, r);
        int64_t x = uniform_below(r[0], (uint32_t)Lx);
        int64_t y = uniform_below(r[1], (uint32_t)Ly);
        int64_t xl = (x + Lx - 1) % Lx, yd = (y + Ly - 1) % Ly;
        uint8_t *sl = &lat[y * Lx + xl], *sc = &lat[y * Lx + x], *sd = &lat[yd * Lx + x];
        int A = bit_to_slope(*sl & 1), B = bit_to_slope(*sc & 1);
        int Cc = bit_to_slope((*sd >> 1) & 1), D = bit_to_slope((*sc >> 1) & 1);
        int kind = site_kind(A, B, Cc, D);
        if (kind == 0) continue;
        int accept = (kind > 0) ? ((uint64_t)r[2] < Tp) : ((uint64_t)r[2] < Tq);
        if (!accept) continue;
        *sl ^= 1; *sc ^= 1; *sd ^= 2; *sc ^= 2;
        if (kind > 0) { if (n_att) (*n_att)++; } else { if (n_det) (*n_det)++; }
        if (x == 0 && y == 0 && H0) *H0 += (kind > 0) ? 2 : -2;
    }
}

/* ------------------------------------------------------------------------ */
/* Heights and the squared width (Sec. I, height reconstruction and Eq.      */
/* (Wdef)).  Reading of the index-garbled reconstruction: the height of      */
/* site (x,y) is h(0,0) plus the sigma_y sum up column 0 to row y plus the   */
/* sigma_x sum along row y to column x:                                      */
/*   h(x,y) = H0 + sum_{k<y} sigma_y(0,k) + sum_{l<x} sigma_x(l,y).          */
/* Writes every height to h (Lx*Ly int64) when h != NULL.                    */
/* ------------------------------------------------------------------------ */
void or_heights(const uint8_t *lat, int64_t Lx, int64_t Ly, int64_t H0, int64_t *h)
{
    int64_t col = H0;
    for (int64_t y = 0; y < Ly; ++y) {
        int64_t hv = col;
        for (int64_t x = 0; x < Lx; ++x) {
            h[y * Lx + x] = hv;
            hv += bit_to_slope(lat[y * Lx + x] & 1);
        }
        col += bit_to_slope((lat[y * Lx + 0] >> 1) & 1);
    }
}

/* S1 = sum h and S2 = sum h^2 over all sites, accumulated exactly in 128-bit
 * integers (Eq. (Wdef): W^2 = S2/N - (S1/N)^2, N = Lx*Ly).  Returns 0, or -1
 * if either sum does not fit a signed 64-bit integer. */
int or_width(const uint8_t *lat, int64_t Lx, int64_t Ly, int64_t H0,
             int64_t *S1, int64_t *S2)
{
    __int128 s1 = 0, s2 = 0;
    int64_t col = H0;
    for (int64_t y = 0; y < Ly; ++y) {
        int64_t hv = col;
        for (int64_t x = 0; x < Lx; ++x) {
            s1 += hv;
            s2 += (__int128)hv * hv;
            hv += bit_to_slope(lat[y * Lx + x] & 1);
        }
        col += bit_to_slope((lat[y * Lx + 0] >> 1) & 1);
    }
    const __int128 lim = ((__int128)1 << 63);
    if (s1 >= lim || s1 < -lim || s2 >= lim) return -1;
    *S1 = (int64_t)s1;
    *S2 = (int64_t)s2;
    return 0;
}

/* S1 and S2 of a band of nrows consecutive rows of a larger lattice, given  */
/* the height h_start of the band's first site (column 0 of its first row): */
/* the same sums as or_width, for a lattice streamed band by band.  Row y of */
/* the band starts at h_start + sum_{k<y} sigma_y(0,k) (column 0 of the band */
/* rows above); the sums come back as 128-bit integers split into a low and */
/* a high 64-bit word (value = hi * 2^64 + lo), and *h_next receives the     */
/* start height of the row after the band.  Rows are summed on host threads. */
void or_width_rows(const uint8_t *rows, int64_t Lx, int64_t nrows, int64_t h_start,
                   uint64_t *s1_lo, int64_t *s1_hi, uint64_t *s2_lo, int64_t *s2_hi,
                   int64_t *h_next)
{
    int64_t *start = (int64_t *)malloc((size_t)(nrows > 0 ? nrows : 1) * sizeof(int64_t));
    int64_t col = h_start;
    for (int64_t y = 0; y < nrows; ++y) {
        start[y] = col;
        col += bit_to_slope((rows[y * Lx + 0] >> 1) & 1);
    }
    *h_next = col;
    __int128 s1 = 0, s2 = 0;
#pragma omp parallel
    {
        __int128 a1 = 0, a2 = 0;
#pragma omp for schedule(static)
        for (int64_t y = 0; y < nrows; ++y) {
            int64_t hv = start[y];
            for (int64_t x = 0; x < Lx; ++x) {
                a1 += hv;
                a2 += (__int128)hv * hv;
                hv += bit_to_slope(rows[y * Lx + x] & 1);
            }
        }
#pragma omp critical
        {
            s1 += a1;
            s2 += a2;
        }
    }
    free(start);
    *s1_lo = (uint64_t)s1;
    *s1_hi = (int64_t)(s1 >> 64);
    *s2_lo = (uint64_t)s2;
    *s2_hi = (int64_t)(s2 >> 64);
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* Number of host threads the block loop of or_sweep may use. */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Ensemble driver for the statistical pins and the random-sequential        */
/* reference of the beta comparison: R independent realizations (seed0 + r)  */
/* from the flat state (Sec. III); after MCS times[i] (strictly increasing,  */
/* >= 1) stores (S1, S2) into out[(r*ntimes + i)*2 + {0,1}].  kind: 0 the     */
/* tiled dynamics with dead cell borders, 1 the random-sequential reference, */
/* 2 the tiled dynamics with delayed cell borders.  Realizations run on      */
/* separate host threads (each realization itself is the plain serial code; */
/* the block loop inside or_sweep then runs on one thread).                  */
/* Returns 0, -1 on a bond conflict, -2 on bad arguments or memory, -3 if a  */
/* width sum leaves int64.                                                   */
/* ------------------------------------------------------------------------ */
int or_ensemble_at(int64_t Lx, int64_t Ly, double p, double q, uint64_t seed0, int64_t R,
                   const int64_t *times, int64_t ntimes, int kind, int64_t *out)
{
    const uint64_t Tp = or_threshold(p), Tq = or_threshold(q);
    for (int64_t i = 0; i < ntimes; ++i)
        if (times[i] < 1 || (i > 0 && times[i] <= times[i - 1])) return -2;
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : rc) if (R > 1)
    for (int64_t r = 0; r < R; ++r) {
        int e = 0; /* this realization's status */
        uint8_t *lat = (uint8_t *)malloc((size_t)(Lx * Ly));
        if (!lat) e = -2;
        else or_flat(lat, Lx, Ly);
        int64_t H0 = 0, t = 0;
        for (int64_t i = 0; i < ntimes && e == 0; ++i) {
            for (; t < times[i] && e == 0; ++t) {
                if (kind == 1)
                    or_rsu_sweep(lat, Lx, Ly, Tp, Tq, seed0 + (uint64_t)r, (uint64_t)t, &H0,
                                 NULL, NULL);
                else if (or_sweep(lat, Lx, Ly, Tp, Tq, seed0 + (uint64_t)r, (uint32_t)t, &H0,
                                  NULL, NULL, 0, kind == 2) != 0)
                    e = -1;
            }
            if (e != 0) break;
            int64_t *o = &out[(r * ntimes + i) * 2];
            if (or_width(lat, Lx, Ly, H0, &o[0], &o[1]) != 0) e = -3;
        }
        free(lat);
        if (e < rc) rc = e; /* the reduction's private copy starts at INT_MAX */
    }
    return rc;
}

/* (S1, S2) after every MCS t = 1..tmax: or_ensemble_at with times 1..tmax. */
int or_ensemble(int64_t Lx, int64_t Ly, double p, double q, uint64_t seed0, int64_t R,
                int64_t tmax, int kind, int64_t *out)
{
    int64_t *times = (int64_t *)malloc((size_t)(tmax > 0 ? tmax : 1) * sizeof(int64_t));
    if (!times) return -2;
    for (int64_t t = 0; t < tmax; ++t) times[t] = t + 1;
    int rc = or_ensemble_at(Lx, Ly, p, q, seed0, R, times, tmax, kind, out);
    free(times);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The tiled dynamics on a window of a larger periodic lattice.  Blocks of a */
/* sweep are independent (Sec. II), so the sites of one block after sweep s  */
/* depend only on that block's sites before it.  Given the exact state of a  */
/* rectangle of the Lx x Ly lattice, a sweep can therefore be applied        */
/* exactly to every block of the sweep's decomposition that lies wholly      */
/* inside the rectangle; the union of those blocks is again a rectangle and  */
/* is where the state is known exactly afterwards.  Starting from a large    */
/* enough rectangle of the flat state, this gives the exact state of any     */
/* part of a lattice far too large to hold, after a few sweeps.              */
/*                                                                          */
/* win: Wx*Wy bytes, win[v*Wx + u] is lattice site ((wx0 + u) mod Lx,        */
/*      (wy0 + v) mod Ly).                                                   */
/* *vx0, *vy0, *vx1, *vy1 (window coordinates, half-open): the rectangle     */
/*      known exactly before the sweep; replaced by the one known after it   */
/*      (empty, vx1 <= vx0, when no block fits).                             */
/* *H0: when lattice site (0,0) lies in a processed block, its height change */
/*      is added (the caller knows whether (0,0) stays inside).              */
/* Needs Wx <= Lx and Wy <= Ly, so a lattice site appears at most once.     */
/* Returns 0, -1 on a bond conflict, -2 on bad arguments.                    */
/* ------------------------------------------------------------------------ */
static int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

int or_window_sweep(uint8_t *win, int64_t Wx, int64_t Wy, int64_t wx0, int64_t wy0,
                    int64_t Lx, int64_t Ly, uint64_t Tp, uint64_t Tq, uint64_t seed,
                    uint32_t s, int64_t *vx0, int64_t *vy0, int64_t *vx1, int64_t *vy1,
                    int64_t *H0, int delayed)
{
    int32_t Bx, By, C;
    if (or_geometry(Lx, Ly, &Bx, &By, &C) != 0 || Wx > Lx || Wy > Ly) return -2;
    int32_t sx, sy;
    or_block_shift(seed, s, Bx, By, &sx, &sy);
    const int64_t nbx = Lx / Bx, nby = Ly / By;
    /* lattice x of window column u is wx0 + u (unwrapped); block column i
     * starts at sx + i*Bx, taken in unwrapped coordinates: the first block
     * starting at or after wx0 + vx0 and the last one ending by wx0 + vx1 */
    const int64_t ax = wx0 + *vx0, bxe = wx0 + *vx1, ay = wy0 + *vy0, bye = wy0 + *vy1;
    const int64_t i0 = floor_div(ax - sx + Bx - 1, Bx), i1 = floor_div(bxe - sx, Bx);
    const int64_t j0 = floor_div(ay - sy + By - 1, By), j1 = floor_div(bye - sy, By);
    if (i1 <= i0 || j1 <= j0) {
        *vx1 = *vx0;
        *vy1 = *vy0;
        return 0;
    }
    int bad = 0;
    int64_t dh = 0;
    const int64_t ni = i1 - i0, nblk = ni * (j1 - j0);
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : dh) reduction(| : bad)
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t i = i0 + b % ni, j = j0 + b / ni;
        const int64_t u0 = sx + i * Bx - wx0, v0 = sy + j * By - wy0; /* window coords */
        const int64_t id = (((j % nby) + nby) % nby) * nbx + (((i % nbx) + nbx) % nbx);
        uint8_t *blk = (uint8_t *)malloc((size_t)Bx * By);
        for (int32_t v = 0; v < By; ++v)
            memcpy(&blk[(size_t)v * Bx], &win[(size_t)(v0 + v) * Wx + u0], (size_t)Bx);
        /* block-local position of lattice site (0,0), if inside this block */
        const int64_t x0 = ((sx + i * Bx) % Lx + Lx) % Lx, y0 = ((sy + j * By) % Ly + Ly) % Ly;
        const int64_t u00 = (Lx - x0) % Lx, v00 = (Ly - y0) % Ly;
        const int32_t su = (u00 < Bx && v00 < By) ? (int32_t)u00 : -1;
        const int32_t sv = (u00 < Bx && v00 < By) ? (int32_t)v00 : -1;
        int64_t h = 0;
        if (or_block_sweep(blk, Bx, By, C, seed, s, (uint32_t)id, Tp, Tq, su, sv, &h, NULL,
                           NULL, NULL, delayed) != 0)
            bad = 1;
        for (int32_t v = 0; v < By; ++v)
            memcpy(&win[(size_t)(v0 + v) * Wx + u0], &blk[(size_t)v * Bx], (size_t)Bx);
        dh += h;
        free(blk);
    }
    if (H0) *H0 += dh;
    *vx0 = sx + i0 * Bx - wx0;
    *vx1 = sx + i1 * Bx - wx0;
    *vy0 = sy + j0 * By - wy0;
    *vy1 = sy + j1 * By - wy0;
    return bad ? -1 : 0;
}
