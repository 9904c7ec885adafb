// Monte Carlo sweep of the octahedron model on gfx950 (Sec. II, Eq. (1)).
//
// One workgroup owns one device-level block per sweep:
//   1. HBM -> LDS: the block's By rows of Bx sites are cut out of the periodic
//      lattice at the sweep's random shift (one-site granularity) with a
//      funnel shift of two stored words per LDS word;
//   2. C*C = 64 steps in LDS: per step one cell origin for the block, one site
//      per 8x8 thread cell, the four-bond test and, when accepted, an XOR of
//      the four slope bits (LDS atomics: neighbouring cells share words but
//      never bits, and XOR commutes);
//   3. LDS -> HBM: the block is written *aligned* into the other lattice copy,
//      whose stored columns start at this sweep's shift.  No two workgroups
//      write the same word, so the store needs no atomics and the shift keeps
//      one-site granularity.
// The height of site (0,0) is tracked without touching the attempt loop: the
// block containing it compares the sigma_x popcount of its row prefix before
// and after the steps (the row's block-border site never moves).
#include "okpz_internal.h"

namespace okpz {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxB = 256;
constexpr int kPitchMax = kMaxB / 32 + 1;              // words per LDS row (+1 pad)
constexpr int kCellsMax = (kMaxB / 8) * (kMaxB / 8);   // 1024 cells of 8x8
constexpr int kCpt = kCellsMax / kThreads;             // cells per thread (max 4)
constexpr int kSteps = 64;                              // C*C with C = 8

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

__device__ __forceinline__ int row_prefix_popc(const uint32_t *row, int n)
{
    int c = 0;
    for (int w = 0; w < (n >> 5); ++w) c += __popc(row[w]);
    if (n & 31) c += __popc(row[n >> 5] & ((1u << (n & 31)) - 1u));
    return c;
}

template <bool kDrawAccept>
__global__ __launch_bounds__(kThreads) void sweep_kernel(SweepLaunch a)
{
    __shared__ uint32_t lds[2 * kMaxB * kPitchMax];
    __shared__ uint8_t origin[kSteps][2];

    const int tid = threadIdx.x;
    const int nblk = a.nbx * a.nby;
    // XCD-aware order: consecutive workgroups are dealt round-robin to the 8
    // XCDs; give each XCD a contiguous run of blocks so neighbouring blocks
    // (which read overlapping words) share that XCD's L2.
    int bid = blockIdx.x;
    if ((nblk & 7) == 0) bid = (blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
    const int bi = bid % a.nbx, bj = bid / a.nbx;
    const int wpr = a.Bx >> 5;
    const int P = wpr + 1;
    const int PL = a.By * P;

    // cell origins of the 64 steps: one counter per pair of steps
    if (tid < kSteps / 2) {
        const Ctr4 r = philox10(Ctr4{a.s, (uint32_t)bid, (uint32_t)tid, kTagOrigin}, a.k0, a.k1);
        origin[2 * tid][0] = (uint8_t)(r.x >> 29);
        origin[2 * tid][1] = (uint8_t)(r.y >> 29);
        origin[2 * tid + 1][0] = (uint8_t)(r.z >> 29);
        origin[2 * tid + 1][1] = (uint8_t)(r.w >> 29);
    }

    // ---- HBM -> LDS with periodic wrap -----------------------------------
    const int x0 = (a.sx + bi * a.Bx) % a.Lx;          // physical first column
    const int xs = (x0 - a.ox_src + a.Lx) % a.Lx;       // its stored column
    const uint32_t off = (uint32_t)(xs & 31);
    const int gw0 = xs >> 5;
    const int y0 = a.sy + bj * a.By;                    // < Ly
    const int nload = 2 * a.By * P;
    for (int e = tid; e < nload; e += kThreads) {
        const int k = e % P;
        const int rest = e / P;
        const int v = rest % a.By;
        const int pl = rest / a.By;
        uint32_t val = 0;
        if (k < wpr) {
            int y = y0 + v;
            if (y >= a.Ly) y -= a.Ly;
            int gw = gw0 + k;
            if (gw >= a.W) gw -= a.W;
            int gw1 = gw + 1;
            if (gw1 == a.W) gw1 = 0;
            const uint32_t *row = a.src + ((size_t)pl * a.Ly + y) * (size_t)a.W;
            val = funnel(row[gw1], row[gw], off);
        }
        lds[pl * PL + v * P + k] = val;
    }
    __syncthreads();

    const bool has00 = (bid == a.blk00);
    int pre00 = 0;
    if (has00 && tid == 0) pre00 = row_prefix_popc(lds + a.v00 * P, a.u00);

    // ---- the thread's cells ----------------------------------------------
    const int ncx = a.Bx >> 3;
    const int ncell = ncx * (a.By >> 3);
    int cxo[kCpt], cyo[kCpt];
    bool live[kCpt];
#pragma unroll
    for (int j = 0; j < kCpt; ++j) {
        const int c = tid + j * kThreads;
        live[j] = c < ncell;
        cxo[j] = (c % ncx) * 8 + 1;
        cyo[j] = (c / ncx) * 8 + 1;
    }
    const int mx = a.Bx - 1, my = a.By - 1;

    for (int g = 0; g < kSteps / 8; ++g) {
        uint32_t sw[kCpt][4];
#pragma unroll
        for (int j = 0; j < kCpt; ++j) {
            const uint32_t c = (uint32_t)(tid + j * kThreads);
            const Ctr4 r = live[j] ? philox10(Ctr4{a.s, (uint32_t)bid, ((uint32_t)g << 16) | c,
                                                   kTagSite},
                                              a.k0, a.k1)
                                   : Ctr4{0, 0, 0, 0};
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
                    const Ctr4 r =
                        live[j] ? philox10(Ctr4{a.s, (uint32_t)bid, ((uint32_t)(k >> 2) << 16) | c,
                                                kTagAccept},
                                           a.k0, a.k1)
                                : Ctr4{0, 0, 0, 0};
                    aw[j][0] = r.x; aw[j][1] = r.y; aw[j][2] = r.z; aw[j][3] = r.w;
                }
            }
            const int ox = origin[k][0], oy = origin[k][1];
#pragma unroll
            for (int j = 0; j < kCpt; ++j) {
                if (!live[j]) continue;
                const uint32_t h16 = (sw[j][e >> 1] >> ((e & 1) * 16)) & 0xffffu;
                const uint32_t i = (h16 * 49u) >> 16;  // one of the 7x7 active sites
                const uint32_t bq = (i * 37u) >> 8;     // i / 7 for i < 49
                const uint32_t aq = i - 7u * bq;
                const int u = (ox + cxo[j] + (int)aq) & mx;
                const int v = (oy + cyo[j] + (int)bq) & my;
                if (u == 0 || v == 0) continue;         // block border: no-op
                uint32_t *rx = lds + v * P;             // sigma_x bits, row v
                uint32_t *ry = lds + PL + v * P;        // sigma_y bits, row v
                const int t = u - 1, w = t >> 5, r = t & 31;
                const uint32_t X = funnel(rx[w + 1], rx[w], (uint32_t)r);  // bx(u-1), bx(u)
                const int wu = u >> 5, ru = u & 31;
                const uint32_t yc = ry[wu] >> ru;       // by(u, v)
                const uint32_t yd = ry[wu - P] >> ru;   // by(u, v-1)
                const uint32_t bc = X >> 1;
                if (((X ^ bc) & (yc ^ yd) & ~(bc ^ yc) & 1u) == 0) continue;
                bool acc;
                if (kDrawAccept)
                    acc = (bc & 1u) ? ((uint64_t)aw[j][e & 3] < a.Tp)
                                    : ((uint64_t)aw[j][e & 3] < a.Tq);
                else
                    acc = (bc & 1u) ? (a.Tp != 0) : (a.Tq != 0);
                if (!acc) continue;
                atomicXor(&rx[w], 3u << r);
                if (r == 31) atomicXor(&rx[w + 1], 1u);
                atomicXor(&ry[wu], 1u << ru);
                atomicXor(&ry[wu - P], 1u << ru);
            }
            __syncthreads();
        }
    }

    if (has00 && tid == 0) {
        const int post00 = row_prefix_popc(lds + a.v00 * P, a.u00);
        *a.h0 += 2 * (int64_t)(post00 - pre00);
    }

    // ---- LDS -> HBM, aligned into the other copy -------------------------
    const int nstore = 2 * a.By * wpr;
    for (int e = tid; e < nstore; e += kThreads) {
        const int k = e % wpr;
        const int rest = e / wpr;
        const int v = rest % a.By;
        const int pl = rest / a.By;
        int y = y0 + v;
        if (y >= a.Ly) y -= a.Ly;
        a.dst[((size_t)pl * a.Ly + y) * (size_t)a.W + (size_t)bi * wpr + k] = lds[pl * PL + v * P + k];
    }
}

}  // namespace

void block_shift(uint32_t k0, uint32_t k1, uint32_t s, const Geometry &g, int32_t *sx, int32_t *sy)
{
    const Ctr4 r = philox10(Ctr4{s, 0, 0, kTagShift}, k0, k1);
    *sx = (int32_t)below(r.x, (uint32_t)g.Bx);
    *sy = (int32_t)below(r.y, (uint32_t)g.By);
}

hipError_t launch_sweep(const SweepLaunch &a, hipStream_t st)
{
    const int nblk = a.nbx * a.nby;
    if (a.need_accept_draws)
        hipLaunchKernelGGL(sweep_kernel<true>, dim3(nblk), dim3(kThreads), 0, st, a);
    else
        hipLaunchKernelGGL(sweep_kernel<false>, dim3(nblk), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace okpz
