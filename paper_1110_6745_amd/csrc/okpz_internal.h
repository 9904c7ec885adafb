// Internal declarations of the okpz HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace okpz {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based bijection
// keyed by the simulation seed, so every random decision of the dynamics is a
// pure function of (seed, counter) and independent of execution order.
struct Ctr4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ Ctr4 philox10(Ctr4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c.z;
        c = Ctr4{(uint32_t)(m1 >> 32) ^ c.y ^ k0, (uint32_t)m1, (uint32_t)(m0 >> 32) ^ c.w ^ k1,
                 (uint32_t)m0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Stream tags (fourth counter word) of the random decisions.
enum : uint32_t { kTagSite = 0, kTagOrigin = 1, kTagShift = 2, kTagAccept = 4 };

// floor(r * n / 2^32): uniform integer below n from a 32-bit draw.
__host__ __device__ __forceinline__ uint32_t below(uint32_t r, uint32_t n)
{
    return (uint32_t)(((uint64_t)r * n) >> 32);
}

// Decomposition geometry of a lattice (Sec. II): block sides and thread cell.
struct Geometry {
    int32_t Bx, By, C;
};

bool geometry_of(int64_t Lx, int64_t Ly, Geometry *g);
uint64_t threshold_of(double prob);

// Device layout of one lattice copy: two bit planes (0 = sigma_x bits,
// 1 = sigma_y bits), each Ly rows of W = Lx/32 words; bit (x' & 31) of word
// (x' >> 5) of row y holds stored column x', where stored column x' is the
// physical column (x' + ox) mod Lx for the copy's offset ox.
struct LatticeView {
    uint32_t *planes;  // 2 * Ly * W words
    int32_t Lx, Ly, W;
    int32_t ox;        // stored-column offset
};

struct SweepLaunch {
    const uint32_t *src;
    uint32_t *dst;
    int64_t *h0;
    int32_t Lx, Ly, W;
    int32_t Bx, By, nbx, nby;
    int32_t ox_src;
    int32_t sx, sy;
    uint32_t s;
    uint32_t k0, k1;
    uint64_t Tp, Tq;
    int32_t blk00, u00, v00;
    int32_t need_accept_draws;
    int32_t delayed_cells;  // 1: delayed thread-cell borders, 0: dead ones
    int32_t in_place;       // 1: one lattice copy (src == dst), blocks stored back in place
    // blocks of this launch: block columns col0 + i col_step, i < ncol, of
    // every block row (launch_sweep sets them; blk00 is then numbered among
    // them, -1 if the block holding site (0,0) is not one of them)
    int32_t col0, col_step, ncol;
};

// Block shift of sweep s (host side; the kernel uses the same values).
void block_shift(uint32_t k0, uint32_t k1, uint32_t s, const Geometry &g, int32_t *sx,
                 int32_t *sy);

hipError_t launch_init(uint32_t *planes, int32_t Ly, int32_t W, hipStream_t st);
// threads per workgroup: 256, 512 or 1024 (execution mapping only; the
// result does not depend on it)
hipError_t launch_sweep(const SweepLaunch &a, int threads, hipStream_t st);
bool sweep_threads_ok(int threads);

}  // namespace okpz
