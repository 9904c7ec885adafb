// Exact squared width of one lattice (Sec. I height reconstruction,
// Eq. (Wdef)) on gfx950: one wavefront per row, then one workgroup combines
// the rows (see width_core.h).
#include "width_core.h"

namespace okpz {
namespace {

constexpr int kRowThreads = 256;
constexpr int kFinalThreads = 1024;

__global__ __launch_bounds__(kRowThreads) void width_rows_kernel(LatticeView v, int64_t *rows)
{
    __shared__ uint32_t lut[256];
    core::width_lut_build(lut);
    __syncthreads();
    const int y = blockIdx.x * (kRowThreads / 64) + (threadIdx.x >> 6);
    if (y >= v.Ly) return;
    core::width_row(v, y, threadIdx.x & 63, lut, rows);
}

__global__ __launch_bounds__(kFinalThreads) void width_final_kernel(const int64_t *rows, int32_t Lx,
                                                                   int32_t Ly, int64_t *out)
{
    __shared__ int64_t lds[64];
    core::width_combine(rows, Lx, Ly, out, lds);
}

}  // namespace

size_t width_scratch_words(int64_t Ly) { return 3 * (size_t)Ly + 4; }

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
    hipLaunchKernelGGL(width_final_kernel, dim3(1), dim3(kFinalThreads), 0, st, rows, v.Lx, v.Ly,
                       out);
    return hipGetLastError();
}

}  // namespace okpz
