// Monte Carlo sweep of the octahedron model on gfx950 (Sec. II, Eq. (1)).
//
// One workgroup owns one device-level block per sweep:
//   1. HBM -> LDS: the block's By rows of Bx sites are cut out of the periodic
//      lattice at the sweep's random shift (one-site granularity; a funnel
//      shift of two stored words per 32 sites) and expanded to one byte per
//      site;
//   2. C*C = 64 steps in LDS: per step one cell origin for the block, one site
//      per 8x8 thread cell, the four-bond test as one table lookup and, when
//      accepted, three byte stores;
//   3. LDS -> HBM: bytes are packed back to bits and the block is written
//      *aligned* into the other lattice copy, whose stored columns start at
//      this sweep's shift.  No two workgroups write the same word, so the
//      store needs no atomics and the shift keeps one-site granularity.
//
// LDS byte of a site: bit 0 = bx (sigma_x = +1), bit 1 = by, bit 2 = block
// border (dead) marker, bit 3 = copy of bx, bit 4 = copy of by.  For the site
// s, its left neighbour l and lower neighbour d, the five-bit code
//   k = (s & 7) | (l & 8) | (d & 16)
// holds bx(u,v), by(u,v), dead(u,v), bx(u-1,v), by(u,v-1).  k = 3 is a local
// minimum (-1 +1; -1 +1), k = 24 a local maximum; a dead site never matches.
// Bit k of a 32-bit table says whether the move is accepted, so the whole
// test is two bit selects and one bit extract.  An accepted move rewrites
// the three bytes (s ^ 0x1B, l ^ 0x09, d ^ 0x12).  Within a step no other lane
// reads or writes those bytes (sites attempted together are never nearest or
// diagonal neighbours: each 8x8 cell has a dead row and column), so plain byte
// stores suffice.
//
// The height of site (0,0) is tracked without touching the attempt loop: the
// block containing it compares the sigma_x count of its row prefix before and
// after the steps (the row's block-border site never moves).
#include "okpz_internal.h"

namespace okpz {
namespace {

constexpr int kMaxB = 256;
// LDS rows are Bx bytes with no padding: for Bx = 256 the bank of a byte
// depends on its column only, so lanes of one cell column collide only when
// they hit the same dword (a broadcast) or rows of one bank dword.
constexpr int kCellsMax = (kMaxB / 8) * (kMaxB / 8);
constexpr int kSteps = 64;                       // C*C with C = 8

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

// 4 bits -> 4 bytes (bit j to bit 0 of byte j)
__device__ __forceinline__ uint32_t spread4(uint32_t nib)
{
    return __umul24(nib, 0x204081u) & 0x01010101u;
}

// 4 bytes with values in bit 0 -> 4 bits, scaled by `w` (byte weights)
__device__ __forceinline__ uint32_t gather4(uint32_t bytes01, uint32_t w, uint32_t acc)
{
    return __builtin_amdgcn_udot4(bytes01, w, acc, false);
}

__device__ __forceinline__ int row_prefix_bx(const uint8_t *row, int n)
{
    int c = 0;
    for (int u = 0; u < n; ++u) c += row[u] & 1;
    return c;
}

// Acceptance modes: p = 1, q = 0 (pure growth, the benchmark's workload);
// p and q each 0 or 1; general p, q (per-attempt acceptance draws).
enum Mode : int { kGrowth = 0, kFixed = 1, kDraw = 2 };

// kFixedB: 256 when the block is 256 x 256 (row pitch known at compile time,
// so the three LDS addresses of an attempt are one register plus immediate
// offsets), 0 for the other block sides (read from the launch arguments).
template <int kThreads, int kMode, int kFixedB>
__global__ __launch_bounds__(kThreads) void sweep_kernel(SweepLaunch a)
{
    constexpr bool kDrawAccept = (kMode == kDraw);
    if (kFixedB) {
        a.Bx = kFixedB;
        a.By = kFixedB;
    }
    constexpr int kCpt = kCellsMax / kThreads;  // cells per thread at 256x256
    // 256 x 256 blocks use a static tile (its base folds into the LDS
    // instruction offsets); other block sides use dynamic LDS.
    extern __shared__ __align__(16) uint8_t smem_dyn[];
    __shared__ __align__(16) uint8_t smem_fix[kFixedB ? (kFixedB + 1) * kFixedB : 16];
    __shared__ uint32_t opack_lds[kSteps / 2];
    uint8_t *smem = kFixedB ? smem_fix : smem_dyn;
    const int pitch = a.Bx;
    uint8_t *tile = smem + pitch;                 // one guard row below row 0

    const int tid = threadIdx.x;
    const int nblk = a.nbx * a.nby;
    // XCD-aware order: consecutive workgroups are dealt round-robin to the 8
    // XCDs; give each XCD a contiguous run of blocks so neighbouring blocks
    // (which read overlapping words) share that XCD's L2.
    int bid = blockIdx.x;
    if ((nblk & 7) == 0) bid = (blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
    const int bi = bid % a.nbx, bj = bid / a.nbx;
    const int wpr = a.Bx >> 5;

    // cell origins of the 64 steps: one counter per pair of steps, computed
    // once per block (thread m: steps 2m, 2m+1, three bits per coordinate);
    // every thread keeps word (lane mod 32) and reads step k's word back with
    // readlane.
    if (tid < kSteps / 2) {
        const Ctr4 r = philox10_dev(Ctr4{a.s, (uint32_t)bid, (uint32_t)tid, kTagOrigin}, a.k0, a.k1);
        opack_lds[tid] = (r.x >> 29) | ((r.y >> 29) << 3) | ((r.z >> 29) << 6) | ((r.w >> 29) << 9);
    }
    // (read after the barrier that ends the load phase)

    // ---- HBM -> LDS with periodic wrap, bits -> bytes ---------------------
    const int x0 = (a.sx + bi * a.Bx) % a.Lx;
    const int xs = (x0 - a.ox_src + a.Lx) % a.Lx;
    const uint32_t off = (uint32_t)(xs & 31);
    const int gw0 = xs >> 5;
    const int y0 = a.sy + bj * a.By;
    for (int e = tid; e < a.By * wpr; e += kThreads) {
        const int k = e % wpr;
        const int v = e / wpr;
        int y = y0 + v;
        if (y >= a.Ly) y -= a.Ly;
        int gw = gw0 + k;
        if (gw >= a.W) gw -= a.W;
        int gw1 = gw + 1;
        if (gw1 == a.W) gw1 = 0;
        const uint32_t *r0 = a.src + (size_t)y * a.W;
        const uint32_t *r1 = a.src + ((size_t)a.Ly + y) * a.W;
        const uint32_t bxw = funnel(r0[gw1], r0[gw], off);
        const uint32_t byw = funnel(r1[gw1], r1[gw], off);
        const uint32_t dead = (v == 0) ? 0x04040404u : 0u;
        uint32_t d[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const uint32_t sx = spread4((bxw >> (4 * m)) & 15u);
            const uint32_t sy = spread4((byw >> (4 * m)) & 15u);
            const uint32_t sxy = sx + (sy << 1);         // bx in bit 0, by in bit 1
            d[m] = sxy + (sxy << 3) + dead;               // copies in bits 3 and 4
        }
        if (k == 0) d[0] |= 4u;  // column u = 0 is the block border
        uint4 *dst = reinterpret_cast<uint4 *>(tile + v * pitch + 32 * k);
        dst[0] = uint4{d[0], d[1], d[2], d[3]};
        dst[1] = uint4{d[4], d[5], d[6], d[7]};
    }
    __syncthreads();

    const uint32_t opack = opack_lds[tid & 31];
    const bool has00 = (bid == a.blk00);
    int pre00 = 0;
    if (has00) {  // uniform per workgroup
        if (tid == 0) pre00 = row_prefix_bx(tile + a.v00 * pitch, a.u00);
        __syncthreads();  // no step may flip that row before it is counted
    }

    // ---- the thread's cells ----------------------------------------------
    // A cell beyond the block's cell count gets zero masks, so its site is
    // always (0,0) of the block, a dead-border site: its attempt is a no-op.
    const int ncx = a.Bx >> 3;
    const int ncell = ncx * (a.By >> 3);
    uint32_t cxo[kCpt], cyo[kCpt], mxj[kCpt], myj[kCpt];
#pragma unroll
    for (int j = 0; j < kCpt; ++j) {
        const int c = tid + j * kThreads;
        const bool live = c < ncell;
        cxo[j] = (uint32_t)((c % ncx) * 8 + 1);
        cyo[j] = (uint32_t)((c / ncx) * 8 + 1);
        mxj[j] = live ? (uint32_t)a.Bx - 1u : 0u;
        myj[j] = live ? (uint32_t)a.By - 1u : 0u;
    }
    // acceptance table: bit 3 = minimum accepted, bit 24 = maximum accepted
    const uint32_t fixed_tbl = (a.Tp != 0 ? (1u << 3) : 0u) | (a.Tq != 0 ? (1u << 24) : 0u);
    (void)fixed_tbl;

    for (int g = 0; g < kSteps / 8; ++g) {
        uint32_t sw[kCpt][4];
#pragma unroll
        for (int j = 0; j < kCpt; ++j) {
            const uint32_t c = (uint32_t)(tid + j * kThreads);
            const Ctr4 r = philox10_dev(Ctr4{a.s, (uint32_t)bid, ((uint32_t)g << 16) | c, kTagSite},
                                        a.k0, a.k1);
            sw[j][0] = r.x; sw[j][1] = r.y; sw[j][2] = r.z; sw[j][3] = r.w;
        }
        uint32_t aw[kCpt][4];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = g * 8 + e;
            if (kDrawAccept && (e & 3) == 0) {
#pragma unroll
                for (int j = 0; j < kCpt; ++j) {
                    const uint32_t c = (uint32_t)(tid + j * kThreads);
                    const Ctr4 r = philox10_dev(
                        Ctr4{a.s, (uint32_t)bid, ((uint32_t)(k >> 2) << 16) | c, kTagAccept}, a.k0,
                        a.k1);
                    aw[j][0] = r.x; aw[j][1] = r.y; aw[j][2] = r.z; aw[j][3] = r.w;
                }
            }
            const uint32_t op = (uint32_t)__builtin_amdgcn_readlane((int)opack, k >> 1) >>
                                (6 * (e & 1));
            const uint32_t ox = op & 7u, oy = (op >> 3) & 7u;
            // all reads of the step first: the cells' byte sets are disjoint
            uint32_t off[kCpt], sv[kCpt], lv[kCpt], dv[kCpt];
#pragma unroll
            for (int j = 0; j < kCpt; ++j) {
                const uint32_t h16 = (e & 1) ? (sw[j][e >> 1] >> 16) : (sw[j][e >> 1] & 0xffffu);
                const uint32_t i = __umul24(h16, 49u) >> 16;  // one of the 7x7 active sites
                const uint32_t bq = __umul24(i, 37u) >> 8;    // i / 7
                const uint32_t ur = ox + cxo[j] + (i - 7u * bq);
                const uint32_t vr = oy + cyo[j] + bq;
                if (kFixedB == 256) {
                    // ((vr mod 256) << 8) | (ur mod 256) in one byte permute
                    off[j] = __builtin_amdgcn_perm(vr, ur, 0x0C0C0400u);
                } else {
                    off[j] = __umul24(vr & myj[j], (uint32_t)pitch) + (ur & mxj[j]);
                }
                sv[j] = smem[off[j] + pitch];
                lv[j] = smem[off[j] + pitch - 1];
                dv[j] = smem[off[j]];
            }
#pragma unroll
            for (int j = 0; j < kCpt; ++j) {
                // five-bit code: bits 0-2 from the site, bit 3 from the left
                // neighbour, bit 4 from the lower neighbour
                // bitwise mux c ? a : b (truth table 0xE4): bit 3 from l,
                // bit 4 from d, the others from s
                const uint32_t t = __builtin_amdgcn_bitop3_b32(lv[j], dv[j], 8u, 0xE4);
                const uint32_t code = __builtin_amdgcn_bitop3_b32(t, sv[j], 24u, 0xE4);
                bool flip;
                if (kMode == kGrowth) {
                    // minimum: the site byte is exactly 0x1B (bx = by = 1 and
                    // copies, not dead) and neither neighbour bit is set
                    const uint32_t m = (lv[j] & 8u) | (dv[j] & ~8u);
                    flip = (((m & 24u) | (sv[j] ^ 0x1Bu)) == 0u);
                } else if (kMode == kFixed) {
                    flip = (fixed_tbl >> code) & 1u;
                } else {
                    const uint32_t r = aw[j][e & 3];
                    const uint32_t tbl = ((uint64_t)r < a.Tp ? (1u << 3) : 0u) |
                                         ((uint64_t)r < a.Tq ? (1u << 24) : 0u);
                    flip = (tbl >> code) & 1u;
                }
                if (flip) {
                    // a growth flip only ever turns 0x1B (minimum) into 0
                    smem[off[j] + pitch] = (kMode == kGrowth) ? (uint8_t)0 : (uint8_t)(sv[j] ^ 0x1Bu);
                    smem[off[j] + pitch - 1] = (uint8_t)(lv[j] ^ 0x09u);
                    smem[off[j]] = (uint8_t)(dv[j] ^ 0x12u);
                }
            }
            __syncthreads();
        }
    }

    if (has00 && tid == 0) {
        const int post00 = row_prefix_bx(tile + a.v00 * pitch, a.u00);
        *a.h0 += 2 * (int64_t)(post00 - pre00);
    }

    // ---- LDS -> HBM: bytes -> bits, aligned into the other copy -----------
    for (int e = tid; e < a.By * wpr; e += kThreads) {
        const int k = e % wpr;
        const int v = e / wpr;
        int y = y0 + v;
        if (y >= a.Ly) y -= a.Ly;
        const uint4 *src = reinterpret_cast<const uint4 *>(tile + v * pitch + 32 * k);
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
        a.dst[(size_t)y * a.W + col] = bxw;
        a.dst[((size_t)a.Ly + y) * a.W + col] = byw;
    }
}

template <int kThreads, int kMode, int kFixedB>
hipError_t launch_b(const SweepLaunch &a, hipStream_t st)
{
    const int nblk = a.nbx * a.nby;
    const size_t lds = kFixedB ? 0 : (size_t)(a.By + 1) * a.Bx;
    static bool attr_set = false;
    if (!attr_set && !kFixedB) {
        // tiles up to 257 x 256 bytes exceed the 64 KiB default of dynamic LDS
        const int cap = (kMaxB + 1) * kMaxB;
        hipError_t e = hipFuncSetAttribute((const void *)sweep_kernel<kThreads, kMode, kFixedB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, cap);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((sweep_kernel<kThreads, kMode, kFixedB>), dim3(nblk), dim3(kThreads), lds,
                       st, a);
    return hipGetLastError();
}

template <int kThreads, int kMode>
hipError_t launch_m(const SweepLaunch &a, hipStream_t st)
{
    if (a.Bx == kMaxB && a.By == kMaxB) return launch_b<kThreads, kMode, kMaxB>(a, st);
    return launch_b<kThreads, kMode, 0>(a, st);
}

template <int kThreads>
hipError_t launch_t(const SweepLaunch &a, hipStream_t st)
{
    const uint64_t one = uint64_t(1) << 32;
    if (a.need_accept_draws) return launch_m<kThreads, kDraw>(a, st);
    if (a.Tp == one && a.Tq == 0) return launch_m<kThreads, kGrowth>(a, st);
    return launch_m<kThreads, kFixed>(a, st);
}

}  // namespace

void block_shift(uint32_t k0, uint32_t k1, uint32_t s, const Geometry &g, int32_t *sx, int32_t *sy)
{
    const Ctr4 r = philox10(Ctr4{s, 0, 0, kTagShift}, k0, k1);
    *sx = (int32_t)below(r.x, (uint32_t)g.Bx);
    *sy = (int32_t)below(r.y, (uint32_t)g.By);
}

bool sweep_threads_ok(int threads) { return threads == 256 || threads == 512 || threads == 1024; }

hipError_t launch_sweep(const SweepLaunch &a, int threads, hipStream_t st)
{
    switch (threads) {
    case 256: return launch_t<256>(a, st);
    case 1024: return launch_t<1024>(a, st);
    default: return launch_t<512>(a, st);
    }
}

}  // namespace okpz
