// Exact squared width from the slope lattice (Sec. I height reconstruction,
// Eq. (Wdef)) on gfx950.
//
// h(x,y) = H0 + G(y) + P_y(x), with G(y) = sum_{k<y} sigma_y(0,k) and
// P_y(x) = sum_{l<x} sigma_x(l,y).  Pass 1 (one wavefront per row): the row's
// words are read once, coalesced, re-aligned to physical columns with a
// funnel shift; each lane turns its word into popcount, a wavefront prefix
// scan gives every word's starting height, and the lane accumulates the
// word's exact sum and sum of squares.  Pass 2 (one workgroup): a scan of the
// column-0 sigma_y bits gives G(y) and the rows are combined into 128-bit
// S1' = sum (h - H0) and S2' = sum (h - H0)^2; the host adds H0 exactly.
#include "okpz_internal.h"

namespace okpz {
namespace {

constexpr int kRowThreads = 256;
constexpr int kFinalThreads = 1024;

__global__ __launch_bounds__(kRowThreads) void width_rows_kernel(LatticeView v, int64_t *rows)
{
    const int lane = threadIdx.x & 63;
    const int y = blockIdx.x * (kRowThreads / 64) + (threadIdx.x >> 6);
    if (y >= v.Ly) return;
    const uint32_t *row = v.planes + (size_t)y * v.W;
    const int xs0 = (v.Lx - v.ox) % v.Lx;  // stored column of physical column 0
    const uint32_t off = (uint32_t)(xs0 & 31);
    const int gws = xs0 >> 5;

    int64_t a1 = 0, a2 = 0;
    int32_t carry = 0;
    for (int base = 0; base < v.W; base += 64) {
        const int k = base + lane;
        uint32_t word = 0;
        int32_t d = 0;
        if (k < v.W) {
            int gw = gws + k;
            if (gw >= v.W) gw -= v.W;
            int gw1 = gw + 1;
            if (gw1 == v.W) gw1 = 0;
            word = __builtin_amdgcn_alignbit(row[gw1], row[gw], off);
            d = 2 * __popc(word) - 32;
        }
        int32_t incl = d;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        const int32_t base_h = carry + incl - d;  // P_y at the word's first site
        if (k < v.W) {
            int32_t q = 0, s1 = 0, s2 = 0;
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                s1 += q;
                s2 += q * q;
                q += (int32_t)((word >> i) & 1u) * 2 - 1;
            }
            const int64_t b = base_h;
            a1 += 32 * b + s1;
            a2 += 32 * b * b + 2 * b * s1 + s2;
        }
        carry += __shfl(incl, 63, 64);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a1 += __shfl_down(a1, o, 64);
        a2 += __shfl_down(a2, o, 64);
    }
    if (lane == 0) {
        const uint32_t *rowy = v.planes + ((size_t)v.Ly + y) * v.W;
        const uint32_t cb = (rowy[xs0 >> 5] >> (xs0 & 31)) & 1u;
        rows[y] = a1;
        rows[(size_t)v.Ly + y] = a2;
        rows[2 * (size_t)v.Ly + y] = (int64_t)cb;
    }
}

__global__ __launch_bounds__(kFinalThreads) void width_final_kernel(const int64_t *rows, int32_t Lx,
                                                                   int32_t Ly, int64_t *out)
{
    __shared__ int32_t scan[kFinalThreads];
    __shared__ int64_t r1[kFinalThreads], r2[kFinalThreads];
    const int tid = threadIdx.x;
    const int per = (Ly + kFinalThreads - 1) / kFinalThreads;
    const int ya = min(Ly, tid * per), yb = min(Ly, ya + per);
    const int64_t *rs1 = rows, *rs2 = rows + Ly, *col = rows + 2 * (size_t)Ly;

    int32_t local = 0;
    for (int y = ya; y < yb; ++y) local += 2 * (int32_t)col[y] - 1;
    scan[tid] = local;
    __syncthreads();
    for (int o = 1; o < kFinalThreads; o <<= 1) {
        const int32_t t = tid >= o ? scan[tid - o] : 0;
        __syncthreads();
        scan[tid] += t;
        __syncthreads();
    }
    int64_t G = scan[tid] - local;  // sum of sigma_y(0,k) for k < ya
    int64_t s1 = 0, s2 = 0;
    for (int y = ya; y < yb; ++y) {
        const int64_t p1 = rs1[y], p2 = rs2[y];
        s1 += (int64_t)Lx * G + p1;
        s2 += (int64_t)Lx * G * G + 2 * G * p1 + p2;
        G += 2 * col[y] - 1;
    }
    r1[tid] = s1;
    r2[tid] = s2;
    __syncthreads();
    if (tid == 0) {
        __int128 t1 = 0, t2 = 0;
        for (int i = 0; i < kFinalThreads; ++i) {
            t1 += r1[i];
            t2 += r2[i];
        }
        out[0] = (int64_t)(uint64_t)t1;
        out[1] = (int64_t)(t1 >> 64);
        out[2] = (int64_t)(uint64_t)t2;
        out[3] = (int64_t)(t2 >> 64);
    }
}

}  // namespace

size_t width_scratch_words(int64_t Ly) { return 3 * (size_t)Ly + 4; }

hipError_t launch_width(const LatticeView &v, int64_t *rows, int64_t *out, hipStream_t st)
{
    const int rpb = kRowThreads / 64;
    hipLaunchKernelGGL(width_rows_kernel, dim3((v.Ly + rpb - 1) / rpb), dim3(kRowThreads), 0, st, v,
                       rows);
    hipLaunchKernelGGL(width_final_kernel, dim3(1), dim3(kFinalThreads), 0, st, rows, v.Lx, v.Ly,
                       out);
    return hipGetLastError();
}

}  // namespace okpz
