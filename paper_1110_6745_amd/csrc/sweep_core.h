// Device side of one Monte Carlo sweep (Sec. II, Eq. (1)) for a group of
// device-level blocks of one lattice; shared by the per-lattice sweep kernel
// and the persistent batch kernel.
//
// A workgroup owns G blocks of one sweep (G = 1 for 256 x 256 blocks, more
// for smaller blocks so that a workgroup always holds about 1024 cells):
//   1. HBM -> LDS: each block's By rows of Bx sites are cut out of the
//      periodic lattice at the sweep's random shift (one-site granularity; a
//      funnel shift of two stored words per 32 sites) and expanded to one byte
//      per site;
//   2. C*C = 64 steps in LDS: per step one cell origin per block, one site per
//      8x8 thread cell, the four-bond test on a five-bit code and, when
//      accepted, three byte stores;
//   3. LDS -> HBM: bytes are packed back to bits and each block is written
//      *aligned* into the other lattice copy, whose stored columns start at
//      this sweep's shift.  No two workgroups write the same word, so the
//      store needs no atomics and the shift keeps one-site granularity.
//
// LDS byte of a site holds the complemented slope bits: bit 0 = nx
// (sigma_x = -1), bit 1 = ny (sigma_y = -1), bit 2 = block border (dead)
// marker, bit 3 = copy of nx, bit 4 = copy of ny.  For the site s, its left
// neighbour l and lower neighbour d, the five-bit code
//   k = (s & 7) | (l & 8) | (d & 16)
// holds nx(u,v), ny(u,v), dead(u,v), nx(u-1,v), ny(u,v-1).  k = 24 is a local
// minimum (-1 +1; -1 +1), k = 3 a local maximum; a dead site never matches.
// A minimum is thus s = 0 with l & 8 and d & 16 set, a test of two bit
// operations.  An accepted move rewrites the three bytes (s ^ 0x1B, l ^ 0x09,
// d ^ 0x12).
// Within a step no other lane reads or writes those bytes (sites attempted
// together are never nearest or diagonal neighbours: each 8x8 cell has a dead
// row and column), so plain byte stores suffice.
//
// The height of site (0,0) is tracked without touching the attempt loop: the
// block containing it compares the sigma_x count of its row prefix before and
// after the steps (the row's block-border site never moves).
#pragma once

#include "okpz_internal.h"

#include <type_traits>

namespace okpz {
namespace core {

constexpr int kMaxB = 256;
constexpr int kCellsMax = (kMaxB / 8) * (kMaxB / 8);  // cells a workgroup holds
constexpr int kSteps = 64;                             // C*C with C = 8
constexpr int kMaxGroup = 64;                          // blocks per group (32 x 32)
constexpr int kPitch = 256;                            // bytes per LDS tile row
// LDS tile of a group, for every block shape: a guard row, then rows of
// kPitch bytes in bands of By rows, each band holding 256 / Bx blocks side by
// side (block g in band g / (256 / Bx), column g mod (256 / Bx)).  Site (u, v)
// of block g sits at byte kPitch + base(g) | v << 8 | u, so an attempt's three
// bytes are one address plus the offsets 256, 255 and 0 whatever the block
// size.  A full group fills the 256 x 256 sites (G Bx By = 65536).  After the
// tile: 33 origin words (32 used; the pad puts the words of consecutive blocks
// in different LDS banks) and 3 placement words per block.
__host__ __device__ inline int tile_bytes(int Bx, int By, int G)
{
    const int bpb = kPitch / Bx;
    return kPitch + ((G + bpb - 1) / bpb) * By * kPitch;
}
constexpr int kGroupLds = kPitch + 65536 + kMaxGroup * 33 * 4 + kMaxGroup * 3 * 4;

// Acceptance modes: p = 1, q = 0 (pure growth); p and q each 0 or 1;
// general p, q (per-attempt acceptance draws).  kDelayedCells added to a
// mode selects the delayed thread-cell borders of Sec. II: every cell draws
// one of its 64 sites, and a step applies the attempts on cell-bulk sites,
// then those on cell edges, then those on cell corners, with a barrier
// after each phase.  kInPlace added to a mode stores the blocks back into
// the copy they were read from (one lattice copy; the launch holds no two
// horizontally adjacent blocks).
enum Mode : int { kGrowth = 0, kFixed = 1, kDraw = 2, kDelayedCells = 4, kInPlace = 8 };

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// Philox4x32-10 with the three-input XORs as single bit operations.
__device__ __forceinline__ Ctr4 philox10_dev(Ctr4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t n0 = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(m1 >> 32), c.y, k0, 0x96);
        const uint32_t n2 = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), c.w, k1, 0x96);
        c = Ctr4{n0, (uint32_t)m1, n2, (uint32_t)m0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Rounds [r0, r1) of Philox4x32-10 on state c (the key of round i is
// (k0 + i W0, k1 + i W1)); rounds 0..9 in order give philox10_dev.
template <int r0, int r1>
__device__ __forceinline__ void philox_rounds(Ctr4 &c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = r0; i < r1; ++i) {
        const uint32_t ka = k0 + (uint32_t)i * 0x9E3779B9u, kb = k1 + (uint32_t)i * 0xBB67AE85u;
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t n0 = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(m1 >> 32), c.y, ka, 0x96);
        const uint32_t n2 = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), c.w, kb, 0x96);
        c = Ctr4{n0, (uint32_t)m1, n2, (uint32_t)m0};
    }
}

// 4 bits -> 4 bytes (bit j to bit 0 of byte j): nib * (1 + 2^7 + 2^14 + 2^21)
// puts bit j at positions j + 7i, all distinct (no carries); byte j keeps
// i = j.
__device__ __forceinline__ uint32_t spread4(uint32_t nib)
{
    return __umul24(nib, 0x204081u) & 0x01010101u;
}

// 4 bytes with values in bit 0 -> 4 bits, scaled by `w` (byte weights)
__device__ __forceinline__ uint32_t gather4(uint32_t bytes01, uint32_t w, uint32_t acc)
{
    return __builtin_amdgcn_udot4(bytes01, w, acc, false);
}

// number of sigma_x = +1 bonds among the first n sites of a tile row
__device__ __forceinline__ int row_prefix_bx(const uint8_t *row, int n)
{
    int c = 0;
    for (int u = 0; u < n; ++u) c += (row[u] & 1) ^ 1;
    return c;
}

__device__ __forceinline__ int ilog2(uint32_t v) { return 31 - __builtin_clz(v); }

// Blocks per group for a block size: about 1024 cells per workgroup.
__host__ __device__ inline int group_size(int Bx, int By, int nblk)
{
    const int cpb = (Bx / 8) * (By / 8);
    int g = kCellsMax / cpb;
    if (g > kMaxGroup) g = kMaxGroup;
    if (g > nblk) g = nblk;
    return g < 1 ? 1 : g;
}

// Eq. (1) on the five-bit code of a site byte s, its left neighbour's byte l
// and its lower neighbour's byte d; r is the attempt's acceptance draw
// (kDraw only).
template <int kMode>
__device__ __forceinline__ bool move_accepted(uint32_t sv, uint32_t lv, uint32_t dv,
                                              uint32_t fixed_tbl, uint32_t r, uint64_t Tp,
                                              uint64_t Tq)
{
    if (kMode == kGrowth) {
        // minimum: s == 0 (nx = ny = 0 and copies, not dead), l & 8 (nx of
        // the left bond) and d & 16 (ny of the lower bond) set:
        // (~l & 8) | (~d & 16) | s == 0, two bit operations (truth table
        // 0xAE: (~A & B) | C)
        const uint32_t t = __builtin_amdgcn_bitop3_b32(lv, 8u, sv, 0xAE);
        return __builtin_amdgcn_bitop3_b32(dv, 16u, t, 0xAE) == 0u;
    }
    // bitwise mux c ? a : b (truth table 0xE4): bit 3 from l, bit 4 from d,
    // the others from s
    const uint32_t t = __builtin_amdgcn_bitop3_b32(lv, dv, 8u, 0xE4);
    const uint32_t code = __builtin_amdgcn_bitop3_b32(t, sv, 24u, 0xE4);
    uint32_t tbl = fixed_tbl;
    if (kMode == kDraw)
        tbl = ((uint64_t)r < Tp ? (1u << 24) : 0u) | ((uint64_t)r < Tq ? (1u << 3) : 0u);
    return (tbl >> code) & 1u;
}

// Set the bits of *w selected by mask to those of v and keep the others; the
// caller guarantees that nobody else writes *w meanwhile.
__device__ __forceinline__ void put_bits(uint32_t *w, uint32_t v, uint32_t mask)
{
    *w = (*w & ~mask) | (v & mask);
}

// LDS atomic XOR of one byte (a 32-bit atomic on the byte's word).
__device__ __forceinline__ void xor_byte(uint8_t *smem, uint32_t off, uint32_t v)
{
    uint32_t *w = reinterpret_cast<uint32_t *>(smem + (off & ~3u));
    atomicXor(w, v << (8 * (off & 3u)));
}

// Origin of the cell grid in step 2m + odd of a block, from the block's
// origin word m (x in byte 2 odd, y in byte 2 odd + 1): x << 16 and y << 16,
// or (y << 16) | x.  A wave-uniform word (kUni) is unpacked with scalar
// shifts; a per-lane word with one byte permute each.
template <bool kUni>
__device__ __forceinline__ uint32_t origin_x16(uint32_t w, int odd)
{
    if (kUni) return odd ? (w & 0x70000u) : ((w << 16) & 0x70000u);
    return __builtin_amdgcn_perm(w, w, odd ? 0x0C020C0Cu : 0x0C000C0Cu);
}
template <bool kUni>
__device__ __forceinline__ uint32_t origin_y16(uint32_t w, int odd)
{
    if (kUni) return odd ? ((w >> 8) & 0x70000u) : ((w << 8) & 0x70000u);
    return __builtin_amdgcn_perm(w, w, odd ? 0x0C030C0Cu : 0x0C010C0Cu);
}
template <bool kUni>
__device__ __forceinline__ uint32_t origin_yx(uint32_t w, int odd)
{
    if (kUni) return odd ? (((w >> 8) & 0x70000u) | ((w >> 16) & 7u)) : (((w << 8) & 0x70000u) | (w & 7u));
    return __builtin_amdgcn_perm(w, w, odd ? 0x0C030C02u : 0x0C010C00u);
}

// One sweep of blocks [b0, b0 + G) of the lattice described by `a`.
//   kFixedB = 256: 256 x 256 blocks, G = 1, static geometry;
//   kFixedB = 0:   block sides 32..256 (powers of two), geometry from `a`.
// Either way the three LDS addresses of an attempt are one register plus
// offsets (the tile layout above).
// kLaneOrg (kFixedB = 0 only): the group's cells are numbered as in one
// 256 x 256 block, so that a wave spans several blocks along a whole tile
// row and each lane fetches its block's origins (the launches use it below
// 128 x 128 sites per block); otherwise the cells of a block are consecutive
// and a wave's 64 cells share a block (needs Bx By >= 4096).
// smem: at least tile_bytes(Bx, By, G) bytes; opk: G * 36 words of LDS
// (origins, then the blocks' placement when kFixedB = 0).
// kStoreThrough: write the new lattice with system-scope stores, which go
// through to memory instead of staying dirty in this XCD's L2 (the persistent
// kernel's hand-over to other XCDs then has little to write back).
template <int kThreads, int kModeFull, int kFixedB, bool kStoreThrough = false, bool kLaneOrg = false>
__device__ __forceinline__ void sweep_group(SweepLaunch a, const int b0, const int G,
                                            uint8_t *__restrict__ smem, uint32_t *opk)
{
    constexpr int kMode = kModeFull & 3;
    constexpr bool kDelayed = (kModeFull & kDelayedCells) != 0;
    constexpr bool kOneCopy = (kModeFull & kInPlace) != 0;
    constexpr bool kDrawAccept = (kMode == kDraw);
    constexpr int kCpt = kCellsMax / kThreads;
    constexpr int kOpkStride = kFixedB ? 32 : 33;  // origin words per block (one block: no pad)
    if (kFixedB) {
        a.Bx = kFixedB;
        a.By = kFixedB;
    }
    // opaque copy of the thread index: in the persistent batch kernel this
    // keeps the compiler from hoisting thread-constant values (counters,
    // cell offsets) out of the work loop, which would pin them in registers
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int Bx = a.Bx, By = a.By;
    const int wpr = Bx >> 5;
    const int lcpb = ilog2((uint32_t)((Bx >> 3) * (By >> 3)));
    const int ncx = Bx >> 3;
    const int lwpr = ilog2((uint32_t)wpr), lby = ilog2((uint32_t)By);
    const int lbpb = 8 - ilog2((uint32_t)Bx);  // 2^lbpb blocks side by side per band
    // offset of block g's first row in the tile, after the guard row
    auto tile_base = [&](int g) -> uint32_t {
        if (kFixedB) return 0u;
        return ((uint32_t)(g >> lbpb) << (8 + lby)) | ((uint32_t)(g & ((1 << lbpb) - 1)) << (8 - lbpb));
    };

    // Block id of group member g.  Groups number the blocks of the launch:
    // all blocks in row-major order, or, for a lattice updated in place, the
    // blocks of the launch's block columns col0, col0 + col_step, ... (ncol
    // of them per block row).
    auto block_id = [&](int g) -> int {
        const int l = b0 + g;
        if (!kOneCopy) return l;
        const int bj = l / a.ncol;
        return bj * a.nbx + a.col0 + (l - bj * a.ncol) * a.col_step;
    };

    // cell origins: one counter per pair of steps and block; word m of block
    // g holds step 2m in bytes 0 (x) and 1 (y), step 2m+1 in bytes 2 and 3
    // (three bits each).
    for (int e = tid; e < G * (kSteps / 2); e += kThreads) {
        const int g = e >> 5, m = e & 31;
        const Ctr4 r = philox10_dev(Ctr4{a.s, (uint32_t)block_id(g), (uint32_t)m, kTagOrigin}, a.k0,
                                    a.k1);
        opk[(e >> 5) * kOpkStride + (e & 31)] = (r.x >> 29) | ((r.y >> 29) << 8) | ((r.z >> 29) << 16) | ((r.w >> 29) << 24);
    }

    // ---- block placement -------------------------------------------------
    // Block bid = block_id(g) starts at lattice site (sx + bi Bx, sy + bj By); that
    // column sits at stored column xs of the source copy.  Per block: xs, the
    // first row and bi (the block's word column in the destination copy).
    auto place = [&](int g, int &xs, int &y0, int &bi) {
        const int bid = block_id(g);
        bi = bid % a.nbx;
        const int bj = bid / a.nbx;
        xs = a.sx + bi * Bx - a.ox_src;
        if (xs < 0) xs += a.Lx;
        y0 = a.sy + bj * By;
    };
    int fxs = 0, fy0 = 0, fbi = 0;
    int *geo = reinterpret_cast<int *>(opk + G * kOpkStride);
    if (kFixedB) {
        place(0, fxs, fy0, fbi);
    } else {
        for (int g = tid; g < G; g += kThreads) {
            int xs, y0, bi;
            place(g, xs, y0, bi);
            geo[3 * g] = xs;
            geo[3 * g + 1] = y0;
            geo[3 * g + 2] = bi;
        }
        __syncthreads();
    }

    // ---- HBM -> LDS with periodic wrap, bits -> bytes ---------------------
    // Element e: tile row R = e >> 3 (band R >> lby, block row v = R mod By)
    // and its 32-site piece c = e & 7 (block c >> lwpr of the band, word
    // k = c mod wpr of the block row): consecutive lanes fill consecutive
    // pieces of a tile row.
    const int nrows = kFixedB ? kFixedB : (((G + (1 << lbpb) - 1) >> lbpb) << lby);
    for (int e = tid; e < nrows * 8; e += kThreads) {
        const int c = e & 7, R = e >> 3;
        const int k = c & (wpr - 1);
        const int v = R & (By - 1);
        const int g = kFixedB ? 0 : (((R >> lby) << lbpb) | (c >> lwpr));
        if (!kFixedB && g >= G) continue;  // the unused end of a last band
        const int xs = kFixedB ? fxs : geo[3 * g];
        int y = (kFixedB ? fy0 : geo[3 * g + 1]) + v;
        if (y >= a.Ly) y -= a.Ly;
        int gw = (xs >> 5) + k;
        if (gw >= a.W) gw -= a.W;
        int gw1 = gw + 1;
        if (gw1 == a.W) gw1 = 0;
        const uint32_t off = (uint32_t)(xs & 31);
        const uint32_t *r0 = a.src + (size_t)y * a.W;
        const uint32_t *r1 = r0 + (size_t)a.Ly * a.W;
        const uint32_t bxw = ~funnel(r0[gw1], r0[gw], off);  // nx bits
        const uint32_t byw = ~funnel(r1[gw1], r1[gw], off);
        uint32_t d[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            // nx in bit 0, ny in bit 1 of each byte (the bit fields are
            // disjoint, so OR composes them); copies in bits 3 and 4
            const uint32_t sxy = spread4((bxw >> (4 * m)) & 15u) |
                                 (__umul24((byw >> (4 * m)) & 15u, 0x408102u) & 0x02020202u);
            d[m] = sxy | (sxy << 3);
        }
        if (v == 0) {  // row v = 0 is the block border (few waves take this)
#pragma unroll
            for (int m = 0; m < 8; ++m) d[m] |= 0x04040404u;
        }
        if (k == 0) d[0] |= 4u;  // column u = 0 is the block border
        uint4 *dst = reinterpret_cast<uint4 *>(smem + kPitch + R * kPitch + 32 * c);
        dst[0] = uint4{d[0], d[1], d[2], d[3]};
        dst[1] = uint4{d[4], d[5], d[6], d[7]};
    }
    __syncthreads();

    // H0: the block holding lattice site (0,0), if it is in this group
    const int g00 = a.blk00 - b0;
    const bool has00 = (g00 >= 0 && g00 < G);  // uniform per workgroup
    int pre00 = 0;
    if (has00) {
        if (tid == 0) pre00 = row_prefix_bx(smem + kPitch + tile_base(g00) + (a.v00 << 8), a.u00);
        __syncthreads();  // no step may flip that row before it is counted
    }

    // ---- the thread's cells ----------------------------------------------
    // A cell beyond the group gets zero masks and tile 0, so its site is
    // always (0,0) of block 0, a dead-border site: its attempt is a no-op.
    const uint32_t mk = ((uint32_t)(By - 1) << 8) | (uint32_t)(Bx - 1);  // (v << 8) | u
    uint32_t cxo[kCpt], cyo[kCpt], mkj[kCpt], gbase[kCpt], cid[kCpt], bidj[kCpt];
    uint32_t gj[kCpt];
    uint32_t opreg[kCpt];
#pragma unroll
    for (int j = 0; j < kCpt; ++j) {
        const int q = tid + j * kThreads;
        int g, c;
        if (kLaneOrg) {
            // cell q at column q mod 32 and row q / 32 of the tile's 32 x 32
            // cells, as in one 256 x 256 block, so that a wave's 64 cells span
            // a whole tile row (all LDS banks) instead of a few neighbouring
            // blocks (fewer banks); with the origin words padded to 33 per
            // block, the blocks a wave then touches read them from different
            // banks
            const int cc = q & 31, cr = q >> 5;
            const int lcx = ilog2((uint32_t)ncx), lcy = lcpb - lcx;
            g = ((cr >> lcy) << lbpb) | (cc >> lcx);
            c = ((cr & ((1 << lcy) - 1)) << lcx) | (cc & (ncx - 1));
        } else {
            g = q >> lcpb;
            c = q & ((1 << lcpb) - 1);
        }
        const bool live = g < G;
        cid[j] = (uint32_t)c;
        bidj[j] = (uint32_t)block_id(live ? g : 0);
        // dead cell borders: the active sites start one in from the origin
        cxo[j] = (uint32_t)((c % ncx) * 8 + (kDelayed ? 0 : 1));
        cyo[j] = (uint32_t)((c / ncx) * 8 + (kDelayed ? 0 : 1));
        mkj[j] = live ? mk : 0u;
        gbase[j] = live ? tile_base(g) : 0u;
        gj[j] = live ? (uint32_t)g : 0u;
        opreg[j] = opk[(live ? g : 0) * kOpkStride + (tid & 31)];
    }
    const uint32_t fixed_tbl = (a.Tp != 0 ? (1u << 24) : 0u) | (a.Tq != 0 ? (1u << 3) : 0u);
    (void)fixed_tbl;

    // Site words of 8 steps come from one Philox call per cell; the call for
    // the next 8 steps is spread over the current ones (about 1.25 rounds
    // per step), where it fills the wait for each step's LDS reads.
    uint32_t sw[kCpt][4];
#pragma unroll
    for (int j = 0; j < kCpt; ++j) {
        const Ctr4 r = philox10_dev(Ctr4{a.s, bidj[j], cid[j], kTagSite}, a.k0, a.k1);
        sw[j][0] = r.x; sw[j][1] = r.y; sw[j][2] = r.z; sw[j][3] = r.w;
    }
    // neighbour bytes: a lane whose site cannot move keeps the bytes it read
    // last (any value gives no move, see below), so no per-step reset is needed
    uint32_t lv[kCpt], dv[kCpt];
#pragma unroll
    for (int j = 0; j < kCpt; ++j) lv[j] = dv[j] = 0;

    // The 64 steps.  kUni: the 64 lanes of a wave share a block, so the
    // origin words are read across lanes into scalar registers; otherwise
    // each lane reads its block's word of the next step pair from LDS during
    // the second step of the current pair.
    auto run_steps = [&](auto uni) __attribute__((always_inline)) {
        constexpr bool kUni = decltype(uni)::value;
        uint32_t opv[kCpt];
        if (!kUni) {
#pragma unroll
            for (int j = 0; j < kCpt; ++j) opv[j] = opk[gj[j] * kOpkStride];
        }
        for (int gs = 0; gs < kSteps / 8; ++gs) {
            Ctr4 nxt[kCpt];
#pragma unroll
            for (int j = 0; j < kCpt; ++j)
                nxt[j] = Ctr4{a.s, bidj[j], ((uint32_t)(gs + 1) << 16) | cid[j], kTagSite};
            uint32_t aw[kCpt][4];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = gs * 8 + e;
                if (kDrawAccept && (e & 3) == 0) {
#pragma unroll
                    for (int j = 0; j < kCpt; ++j) {
                        const Ctr4 r = philox10_dev(
                            Ctr4{a.s, bidj[j], ((uint32_t)(k >> 2) << 16) | cid[j], kTagAccept}, a.k0,
                            a.k1);
                        aw[j][0] = r.x; aw[j][1] = r.y; aw[j][2] = r.z; aw[j][3] = r.w;
                    }
                }
                // all reads of the step first: the cells' byte sets are disjoint.
                // For a site byte that is neither 0 nor 0x1B the low three bits
                // of the site byte already rule out a move, whatever the
                // neighbour bytes hold.
                uint32_t off[kCpt], sv[kCpt], phs[kCpt];
#pragma unroll
                for (int j = 0; j < kCpt; ++j) {
                    if (kUni && (e & 1) == 0) opv[j] = (uint32_t)__builtin_amdgcn_readlane((int)opreg[j], k >> 1);
                    const uint32_t h16 = (e & 1) ? (sw[j][e >> 1] >> 16) : (sw[j][e >> 1] & 0xffffu);
                    uint32_t o;
                    if (kDelayed) {
                        // site i = floor(64 h / 2^16) of the 8 x 8 cell: a = i mod 8,
                        // b = i div 8; phase 0 bulk, 1 edge (one of a, b zero),
                        // 2 corner
                        const uint32_t ca = (h16 >> 10) & 7u, cb = h16 >> 13;
                        phs[j] = (uint32_t)(ca == 0u) + (uint32_t)(cb == 0u);
                        // row in the high half, column in the low half (no
                        // carry between them); one byte permute takes both
                        // mod 256 into (row << 8) | column
                        const uint32_t Y = ((cb << 16) | ca) + ((cyo[j] << 16) | cxo[j]) +
                                           origin_yx<kUni>(opv[j], e & 1);
                        o = __builtin_amdgcn_perm(Y, Y, 0x0C0C0200u);
                    } else {
                        // Active site i = floor(49 h / 2^16) of the 7 x 7 (row-major),
                        // split as i = 7 q + a without a division: with 7 h = q 2^16 + r,
                        // q = floor(7 h / 2^16) = i div 7 and a = floor(7 r / 2^16) = i mod 7.
                        // Y = 7 h + (row base << 16) keeps r in its low half, so
                        // bits 16..23 of Y and X are the row and the column mod
                        // 256; one byte permute packs them into (row << 8) | column
                        const uint32_t Y = __umul24(h16, 7u) + (cyo[j] << 16) + origin_y16<kUni>(opv[j], e & 1);
                        const uint32_t X =
                            __umul24(Y & 0xffffu, 7u) + (cxo[j] << 16) + origin_x16<kUni>(opv[j], e & 1);
                        o = __builtin_amdgcn_perm(Y, X, 0x0C0C0602u);
                    }
                    // smaller blocks: row and column mod the block sides, then
                    // the block's place in the tile (disjoint bits)
                    if (!kFixedB) o = (o & mkj[j]) | gbase[j];
                    off[j] = o;
                    sv[j] = smem[off[j] + kPitch];
                    // behind the site read of a pair's second step: the next
                    // pair's origin word (the last pair reads its own again)
                    if (!kUni && (e & 1) == 1) opv[j] = opk[gj[j] * kOpkStride + min((k >> 1) + 1, kSteps / 2 - 1)];
                }
                // While the reads are in flight: this step's share of the next
                // Philox call, pinned here so that it is not sunk to its use.
                // It is filler work: at low wave priority, so that waves whose
                // step chain can go on (towards the step barrier) issue first.
                __builtin_amdgcn_s_setprio(0);
                if (gs + 1 < kSteps / 8) {
#pragma unroll
                    for (int j = 0; j < kCpt; ++j) {
                        switch (e) {  // rounds 0,1 | 1,2 | 2,3 | 3,5 | 5,6 | 6,7 | 7,8 | 8,10
                        case 0: philox_rounds<0, 1>(nxt[j], a.k0, a.k1); break;
                        case 1: philox_rounds<1, 2>(nxt[j], a.k0, a.k1); break;
                        case 2: philox_rounds<2, 3>(nxt[j], a.k0, a.k1); break;
                        case 3: philox_rounds<3, 5>(nxt[j], a.k0, a.k1); break;
                        case 4: philox_rounds<5, 6>(nxt[j], a.k0, a.k1); break;
                        case 5: philox_rounds<6, 7>(nxt[j], a.k0, a.k1); break;
                        case 6: philox_rounds<7, 8>(nxt[j], a.k0, a.k1); break;
                        default: philox_rounds<8, 10>(nxt[j], a.k0, a.k1); break;
                        }
                        asm volatile("" : "+v"(nxt[j].x), "+v"(nxt[j].y), "+v"(nxt[j].z), "+v"(nxt[j].w));
                    }
                }
                __builtin_amdgcn_s_setprio(2);
                if (kDelayed) {
                    // Three phases.  Within one, attempted sites are never nearest
                    // neighbours.  Bulk sites are not diagonal neighbours either
                    // (as in the dead-border steps), and corners are 8 apart, so
                    // plain byte stores suffice there; an edge site and the edge
                    // site diagonally up and to the left of it (the next cell's
                    // bottom row) can share a neighbour byte, so edge flips are
                    // atomic XORs (plain stores with atomics for that pair only
                    // measured slower: 30.8 against 26.4 ms at 2^17).
                    // Every phase uses the site byte read above: a site's own byte
                    // changes only by a move at the site, at its right neighbour
                    // or at its upper neighbour.  For a bulk site those are its
                    // own cell's sites or a later-phase site of the next cell
                    // (edge); for an edge site, its own cell's or the next
                    // cell's corner; for a corner, its own cell's.  A cell
                    // attempts one site per step, so no move of an earlier
                    // phase touches the byte of a later-phase site.
#pragma unroll
                    for (int ph = 0; ph < 3; ++ph) {
#pragma unroll
                        for (int j = 0; j < kCpt; ++j) {
                            if (phs[j] != (uint32_t)ph) continue;
                            const uint32_t s0 = sv[j];
                            if (s0 != 0u && (kMode == kGrowth || s0 != 0x1Bu)) continue;
                            uint32_t l0 = smem[off[j] + kPitch - 1];
                            uint32_t d0 = smem[off[j]];
                            // the loads zero-extend; as in the dead-border steps,
                            // keep the code generator from re-masking the bytes
                            asm volatile("" : "+v"(l0), "+v"(d0));
                            const uint32_t r = kDrawAccept ? aw[j][e & 3] : 0u;
                            if (!move_accepted<kMode>(s0, l0, d0, fixed_tbl, r, a.Tp, a.Tq)) continue;
                            if (ph == 1) {
                                xor_byte(smem, off[j] + kPitch, 0x1Bu);
                                xor_byte(smem, off[j] + kPitch - 1, 0x09u);
                                xor_byte(smem, off[j], 0x12u);
                            } else {
                                smem[off[j] + kPitch] = (uint8_t)(s0 ^ 0x1Bu);
                                smem[off[j] + kPitch - 1] = (uint8_t)(l0 ^ 0x09u);
                                smem[off[j]] = (uint8_t)(d0 ^ 0x12u);
                            }
                        }
                        __syncthreads();
                    }
                    continue;
                }
#pragma unroll
                for (int j = 0; j < kCpt; ++j) {
                    // the loads zero-extend; keep the code generator from
                    // re-narrowing the bytes (it would add masking operations)
                    asm volatile("" : "+v"(sv[j]));
                    // Only a site at a local minimum (byte 0) or maximum (0x1B)
                    // can move; only those lanes read the two neighbour bytes,
                    // which roughly halves the LDS read traffic of a step.
                    const bool cand = (sv[j] == 0u) || (kMode != kGrowth && sv[j] == 0x1Bu);
                    if (cand) {
                        lv[j] = smem[off[j] + kPitch - 1];
                        dv[j] = smem[off[j]];
                    }
                    asm volatile("" : "+v"(lv[j]), "+v"(dv[j]));
                }
#pragma unroll
                for (int j = 0; j < kCpt; ++j) {
                    const uint32_t r = kDrawAccept ? aw[j][e & 3] : 0u;
                    if (move_accepted<kMode>(sv[j], lv[j], dv[j], fixed_tbl, r, a.Tp, a.Tq)) {
                        // a growth flip only ever turns 0 (minimum) into 0x1B
                        smem[off[j] + kPitch] = (kMode == kGrowth) ? (uint8_t)0x1Bu : (uint8_t)(sv[j] ^ 0x1Bu);
                        smem[off[j] + kPitch - 1] = (uint8_t)(lv[j] ^ 0x09u);
                        smem[off[j]] = (uint8_t)(dv[j] ^ 0x12u);
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int j = 0; j < kCpt; ++j) {
                sw[j][0] = nxt[j].x; sw[j][1] = nxt[j].y; sw[j][2] = nxt[j].z; sw[j][3] = nxt[j].w;
            }
        }
    };
    run_steps(std::integral_constant<bool, kFixedB != 0 || !kLaneOrg>{});

    // the store below is not on any step's critical path: back to low
    // priority, behind the steps of a co-resident workgroup
    __builtin_amdgcn_s_setprio(0);

    if (has00 && tid == 0) {
        const int post00 = row_prefix_bx(smem + kPitch + tile_base(g00) + (a.v00 << 8), a.u00);
        *a.h0 += 2 * (int64_t)(post00 - pre00);
    }

    // ---- LDS -> HBM: bytes -> bits, aligned into the other copy -----------
    // (elements as in the load above)
    for (int e = tid; e < nrows * 8; e += kThreads) {
        const int c = e & 7, R = e >> 3;
        const int k = c & (wpr - 1);
        const int v = R & (By - 1);
        const int g = kFixedB ? 0 : (((R >> lby) << lbpb) | (c >> lwpr));
        if (!kFixedB && g >= G) continue;
        const int bi = kFixedB ? fbi : geo[3 * g + 2];
        int y = (kFixedB ? fy0 : geo[3 * g + 1]) + v;
        if (y >= a.Ly) y -= a.Ly;
        const uint4 *src = reinterpret_cast<const uint4 *>(smem + kPitch + R * kPitch + 32 * c);
        const uint4 q0 = src[0], q1 = src[1];
        const uint32_t d[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
        uint32_t bxw = 0, byw = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {  // byte b of the word: sites 8b .. 8b+7
            const uint32_t lo = d[2 * b], hi = d[2 * b + 1];
            const uint32_t xb = gather4(hi & 0x01010101u, 0x80402010u,
                                        gather4(lo & 0x01010101u, 0x08040201u, 0u));
            const uint32_t yb = gather4((hi >> 1) & 0x01010101u, 0x80402010u,
                                        gather4((lo >> 1) & 0x01010101u, 0x08040201u, 0u));
            bxw |= xb << (8 * b);
            byw |= yb << (8 * b);
        }
        const size_t col = (size_t)bi * wpr + k;
        if (kOneCopy) {
            // One lattice copy: the block goes back where it was read from,
            // its row segment starting at stored column xs (off = xs mod 32
            // is the same for every block of the sweep).  Blocks cover
            // disjoint sites and a block reads and writes only its own, so no
            // block sees another's update.  Segment word k takes tile word k
            // shifted up by off plus the top off bits of tile word k-1 (the
            // previous lane's).  The segment's first and one-past-last words
            // are shared with the left and right neighbour blocks, which the
            // host never puts in the same launch, so a plain read-modify-write
            // replaces only this block's bits.  With one block per row those
            // two words are one word, all of it this block's: the first lane
            // writes it whole, with the last lane's top bits.
            const int xs = kFixedB ? fxs : geo[3 * g];
            const uint32_t off = (uint32_t)(xs & 31);
            const uint32_t nx = ~bxw, ny = ~byw;
            const uint32_t px = __shfl_up(nx, 1, 64), py = __shfl_up(ny, 1, 64);
            const uint32_t lx = __shfl_down(nx, wpr - 1, 64), ly = __shfl_down(ny, wpr - 1, 64);
            uint32_t *rx = a.dst + (size_t)y * a.W, *ry = a.dst + ((size_t)a.Ly + y) * a.W;
            int gw = (xs >> 5) + k;
            if (gw >= a.W) gw -= a.W;
            if (off == 0) {
                rx[gw] = nx;
                ry[gw] = ny;
            } else if (k != 0) {
                rx[gw] = (nx << off) | (px >> (32 - off));
                ry[gw] = (ny << off) | (py >> (32 - off));
            } else if (a.nbx == 1) {
                rx[gw] = (nx << off) | (lx >> (32 - off));
                ry[gw] = (ny << off) | (ly >> (32 - off));
            } else {
                put_bits(rx + gw, nx << off, ~0u << off);
                put_bits(ry + gw, ny << off, ~0u << off);
            }
            if (k == wpr - 1 && off != 0 && a.nbx != 1) {
                int gl = gw + 1;
                if (gl == a.W) gl = 0;
                put_bits(rx + gl, nx >> (32 - off), (1u << off) - 1u);
                put_bits(ry + gl, ny >> (32 - off), (1u << off) - 1u);
            }
            continue;
        }
        uint32_t *w0 = a.dst + (size_t)y * a.W + col, *w1 = a.dst + ((size_t)a.Ly + y) * a.W + col;
        if (kStoreThrough) {
            __hip_atomic_store(w0, ~bxw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(w1, ~byw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        } else {
            *w0 = ~bxw;  // back to sigma = +1 bits
            *w1 = ~byw;
        }
    }
}

}  // namespace core
}  // namespace okpz
