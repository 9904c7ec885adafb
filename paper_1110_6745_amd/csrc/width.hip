// Exact squared width of one lattice (Sec. I height reconstruction,
// Eq. (Wdef)) on gfx950: one wavefront per row (width_core.h), then a
// two-level combine of the rows into the 128-bit sums.
//
// Rows y of block b (kBlockRows consecutive rows) have G(y) = G_b + g(y) with
// g the prefix of the column-0 sigma_y inside the block, so
//   sum_b-rows (Lx G + p1)                = n_b Lx G_b + A_b,
//   sum_b-rows (Lx G^2 + 2 G p1 + p2)     = n_b Lx G_b^2 + 2 G_b A_b + B_b,
// with A_b = sum (Lx g + p1), B_b = sum (Lx g^2 + 2 g p1 + p2).  Every block
// writes (delta_b, A_b, B_b) with delta_b its sigma_y sum; one workgroup scans
// the delta_b into G_b and adds the blocks up.  Up to kOneGroupRows rows one
// workgroup combines the rows directly (one launch less, which is what a
// small lattice's measurement costs).
#include "width.h"
#include "width_core.h"

namespace okpz {
namespace {

constexpr int kRowThreads = 256;
constexpr int kBlockRows = 256;
constexpr int kTotalThreads = 1024;
constexpr int kOneGroupRows = 8192;

__global__ __launch_bounds__(kRowThreads) void width_rows_kernel(LatticeView v, int64_t *rows)
{
    __shared__ uint32_t lut[256];
    core::width_lut_build(lut);
    __syncthreads();
    const int y = blockIdx.x * (kRowThreads / 64) + (threadIdx.x >> 6);
    if (y >= v.Ly) return;
    core::width_row(v, y, threadIdx.x & 63, lut, rows);
}

__global__ __launch_bounds__(kTotalThreads) void width_final_kernel(const int64_t *rows, int32_t Lx,
                                                                    int32_t Ly, int64_t *out)
{
    __shared__ int64_t lds[64];
    core::width_combine(rows, Lx, Ly, out, lds);
}

// blk[4 b ..] = {delta_b, A_b, B_b lo, B_b hi} of rows [b kBlockRows, ...).
__global__ __launch_bounds__(kBlockRows) void width_blocks_kernel(const int64_t *rows, int32_t Lx,
                                                                  int32_t Ly, int64_t *blk)
{
    __shared__ int64_t lds[32];
    const int y = blockIdx.x * kBlockRows + threadIdx.x;
    const bool in = y < Ly;
    const int64_t d = in ? 2 * rows[2 * (size_t)Ly + y] - 1 : 0;
    int64_t delta;
    const int64_t g = core::block_exclusive_scan(d, lds, &delta);
    const int64_t p1 = in ? rows[y] : 0, p2 = in ? rows[(size_t)Ly + y] : 0;
    const __int128 a = in ? (__int128)Lx * g + p1 : 0;
    const __int128 b = in ? (__int128)Lx * g * g + 2 * (__int128)g * p1 + p2 : 0;
    const __int128 A = core::block_sum_i128(a, lds);
    const __int128 B = core::block_sum_i128(b, lds);
    if (threadIdx.x == 0) {
        int64_t *o = blk + 4 * (size_t)blockIdx.x;
        o[0] = delta;
        o[1] = (int64_t)A;
        o[2] = (int64_t)(uint64_t)B;
        o[3] = (int64_t)(uint64_t)((unsigned __int128)B >> 64);
    }
}

// out[0..3] = {S1' lo, S1' hi, S2' lo, S2' hi} from the nb block records.
__global__ __launch_bounds__(kTotalThreads) void width_total_kernel(const int64_t *blk, int32_t nb,
                                                                    int32_t Lx, int32_t Ly,
                                                                    int64_t *out)
{
    __shared__ int64_t lds[32];
    const int per = (nb + kTotalThreads - 1) / kTotalThreads;
    const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
    int64_t local = 0;
    for (int b = b0; b < b1; ++b) local += blk[4 * (size_t)b];
    int64_t unused;
    int64_t G = core::block_exclusive_scan(local, lds, &unused);
    __int128 s1 = 0, s2 = 0;
    for (int b = b0; b < b1; ++b) {
        const int64_t *r = blk + 4 * (size_t)b;
        const __int128 nL = (__int128)min(kBlockRows, Ly - b * kBlockRows) * Lx;
        const __int128 A = r[1];
        const __int128 B = (__int128)(((unsigned __int128)(uint64_t)r[3] << 64) | (uint64_t)r[2]);
        s1 += nL * G + A;
        s2 += nL * G * G + 2 * (__int128)G * A + B;
        G += r[0];
    }
    const __int128 S1 = core::block_sum_i128(s1, lds);
    const __int128 S2 = core::block_sum_i128(s2, lds);
    if (threadIdx.x == 0) {
        out[0] = (int64_t)(uint64_t)S1;
        out[1] = (int64_t)(uint64_t)((unsigned __int128)S1 >> 64);
        out[2] = (int64_t)(uint64_t)S2;
        out[3] = (int64_t)(uint64_t)((unsigned __int128)S2 >> 64);
    }
}

int32_t width_blocks(int64_t Ly) { return (int32_t)((Ly + kBlockRows - 1) / kBlockRows); }

}  // namespace

size_t width_scratch_words(int64_t Ly) { return 3 * (size_t)Ly + 4 * (size_t)width_blocks(Ly) + 4; }

hipError_t launch_width_rows(const LatticeView &v, int64_t *rows, hipStream_t st)
{
    const int rpb = kRowThreads / 64;
    hipLaunchKernelGGL(width_rows_kernel, dim3((v.Ly + rpb - 1) / rpb), dim3(kRowThreads), 0, st, v,
                       rows);
    return hipGetLastError();
}

hipError_t launch_width(const LatticeView &v, int64_t *rows, int64_t *out, hipStream_t st)
{
    const hipError_t e = launch_width_rows(v, rows, st);
    if (e != hipSuccess) return e;
    if (v.Ly <= kOneGroupRows) {
        hipLaunchKernelGGL(width_final_kernel, dim3(1), dim3(kTotalThreads), 0, st, rows, v.Lx, v.Ly,
                           out);
        return hipGetLastError();
    }
    const int32_t nb = width_blocks(v.Ly);
    int64_t *blk = rows + 3 * (size_t)v.Ly;
    hipLaunchKernelGGL(width_blocks_kernel, dim3(nb), dim3(kBlockRows), 0, st, rows, v.Lx, v.Ly,
                       blk);
    hipLaunchKernelGGL(width_total_kernel, dim3(1), dim3(kTotalThreads), 0, st, blk, nb, v.Lx, v.Ly,
                       out);
    return hipGetLastError();
}

}  // namespace okpz
