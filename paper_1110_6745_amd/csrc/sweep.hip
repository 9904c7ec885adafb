// Per-lattice Monte Carlo sweep kernel on gfx950 (Sec. II, Eq. (1)): one
// workgroup per group of device-level blocks (see sweep_core.h), one launch
// per MCS.
#include "sweep_core.h"

namespace okpz {
namespace {

using core::kDraw;
using core::kFixed;
using core::kGrowth;

// Groups per launch: a grid dimension holds fewer than 2^32 work-items, so
// the sweep of a lattice above 2^18 x 2^18 sites takes several launches
// (blocks are independent within a sweep; the order does not matter).
constexpr int kMaxGroupsPerLaunch = 1 << 21;

template <int kThreads, int kMode, int kFixedB, bool kLaneOrg>
__global__ __launch_bounds__(kThreads) void sweep_kernel(SweepLaunch a, int G, int g0)
{
    // Static LDS, so that the tile's base folds into the LDS instruction
    // offsets: one 256 x 256 block, or a group of smaller blocks with their
    // origin and placement words.
    __shared__ __align__(16) uint8_t smem_fix[kFixedB ? core::kPitch + kFixedB * core::kPitch : core::kGroupLds];
    __shared__ uint32_t opk_fix[kFixedB ? 32 : 1];
    const int nblk = a.ncol * a.nby;
    const int nl = gridDim.x;  // groups of this launch, starting at group g0
    // XCD-aware order: consecutive workgroups are dealt round-robin to the 8
    // XCDs; give each XCD a contiguous run of groups so neighbouring blocks
    // (which read overlapping words) share that XCD's L2.
    int gid = blockIdx.x;
    if ((nl & 7) == 0) gid = (blockIdx.x & 7) * (nl >> 3) + (blockIdx.x >> 3);
    gid += g0;
    const int b0 = gid * G;
    const int Gc = min(G, nblk - b0);
    if (kFixedB) {
        core::sweep_group<kThreads, kMode, kFixedB>(a, b0, 1, smem_fix, opk_fix);
    } else {
        const int tiles = core::tile_bytes(a.Bx, a.By, Gc);
        core::sweep_group<kThreads, kMode, kFixedB, false, kLaneOrg>(
            a, b0, Gc, smem_fix, reinterpret_cast<uint32_t *>(smem_fix + tiles));
    }
}

template <int kThreads, int kMode, int kFixedB, bool kLaneOrg>
hipError_t launch_b(const SweepLaunch &a, hipStream_t st)
{
    const int nblk = a.ncol * a.nby;
    const int G = kFixedB ? 1 : core::group_size(a.Bx, a.By, nblk);
    const int ngroups = (nblk + G - 1) / G;
    for (int g0 = 0; g0 < ngroups; g0 += kMaxGroupsPerLaunch) {
        const int n = ngroups - g0 < kMaxGroupsPerLaunch ? ngroups - g0 : kMaxGroupsPerLaunch;
        hipLaunchKernelGGL((sweep_kernel<kThreads, kMode, kFixedB, kLaneOrg>), dim3(n), dim3(kThreads), 0,
                           st, a, G, g0);
    }
    return hipGetLastError();
}

template <int kThreads, int kMode>
hipError_t launch_m(const SweepLaunch &a, hipStream_t st)
{
    if (a.Bx == core::kMaxB && a.By == core::kMaxB) return launch_b<kThreads, kMode, core::kMaxB, false>(a, st);
    // blocks of 256 cells or more: a wave's cells share a block; smaller ones
    // spread a wave over a whole tile row (per-lane origins)
    if (a.Bx * a.By >= 128 * 128) return launch_b<kThreads, kMode, 0, false>(a, st);
    return launch_b<kThreads, kMode, 0, true>(a, st);
}

template <int kThreads, int kCells>
hipError_t launch_c(const SweepLaunch &a, hipStream_t st)
{
    const uint64_t one = uint64_t(1) << 32;
    if (a.need_accept_draws) return launch_m<kThreads, kDraw | kCells>(a, st);
    if (a.Tp == one && a.Tq == 0) return launch_m<kThreads, kGrowth | kCells>(a, st);
    return launch_m<kThreads, kFixed | kCells>(a, st);
}

template <int kThreads>
hipError_t launch_t(const SweepLaunch &a, hipStream_t st)
{
    if (a.in_place) {
        if (a.delayed_cells) return launch_c<kThreads, core::kDelayedCells | core::kInPlace>(a, st);
        return launch_c<kThreads, core::kInPlace>(a, st);
    }
    if (a.delayed_cells) return launch_c<kThreads, core::kDelayedCells>(a, st);
    return launch_c<kThreads, 0>(a, st);
}

}  // namespace

void block_shift(uint32_t k0, uint32_t k1, uint32_t s, const Geometry &g, int32_t *sx, int32_t *sy)
{
    const Ctr4 r = philox10(Ctr4{s, 0, 0, kTagShift}, k0, k1);
    *sx = (int32_t)below(r.x, (uint32_t)g.Bx);
    *sy = (int32_t)below(r.y, (uint32_t)g.By);
}

bool sweep_threads_ok(int threads) { return threads == 256 || threads == 512 || threads == 1024; }

namespace {

hipError_t launch_threads(const SweepLaunch &a, int threads, hipStream_t st)
{
    switch (threads) {
    case 256: return launch_t<256>(a, st);
    case 512: return launch_t<512>(a, st);
    default: return launch_t<1024>(a, st);
    }
}

}  // namespace

hipError_t launch_sweep(const SweepLaunch &a, int threads, hipStream_t st)
{
    SweepLaunch b = a;
    if (!a.in_place || a.nbx == 1) {
        b.col0 = 0;
        b.col_step = 1;
        b.ncol = a.nbx;
        return launch_threads(b, threads, st);
    }
    // One copy updated in place: horizontally adjacent blocks share a word
    // at either end of each row segment, so they go to different launches:
    // even block columns, odd ones, and with an odd count the last column
    // (the left neighbour of column 0) on its own.
    const int odd = a.nbx & 1;
    const int cls[3][3] = {{0, 2, a.nbx / 2}, {1, 2, a.nbx / 2}, {a.nbx - 1, 1, 1}};
    const int bi00 = a.blk00 % a.nbx, bj00 = a.blk00 / a.nbx;
    for (int c = 0; c < 2 + odd; ++c) {
        b.col0 = cls[c][0];
        b.col_step = cls[c][1];
        b.ncol = cls[c][2];
        const int i = bi00 - b.col0;
        const bool mine = i >= 0 && i % b.col_step == 0 && i / b.col_step < b.ncol;
        b.blk00 = mine ? bj00 * b.ncol + i / b.col_step : -1;
        const hipError_t e = launch_threads(b, threads, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace okpz
