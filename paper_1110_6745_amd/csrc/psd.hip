// Power spectrum density of the surface along the lattice axes (Sec. III,
// Eqs. (PSD) and (hF)) on gfx950.
//
// For k = (2 pi n / Lx, 0) the transform of Eq. (hF) only sees the column
// sums of the heights, and for k = (0, 2 pi n / Ly) only the row sums:
//   h(k) = (Lx Ly)^{-1/2} sum_x e^{i k x} (X(x) - <X>),  X(x) = sum_y h(x,y).
// With h(x,y) = H0 + G(y) + P_y(x) (Sec. I reconstruction), up to constants
// that drop out of every n > 0,
//   X(x) = sum_{l<x} (2 c(l) - Ly),  c(l) = number of rows with sigma_x(l,y) = +1,
//   Y(y) = Lx G(y) + sum_x P_y(x).
// So the surface is reduced exactly, in integers, to two profiles: a column
// popcount of the sigma_x plane (one pass over N/8 bytes) and the per-row sums
// the width pass already makes.  Each profile, minus its mean, goes through a
// radix-2 decimation-in-frequency FFT in fp64: global passes while a
// butterfly's span exceeds the LDS tile, then one LDS-resident pass per tile;
// the output stays in bit-reversed order and the spectrum kernel reads it so.
#include "width_core.h"

namespace okpz {
namespace {

constexpr int kCountThreads = 256;
constexpr int kScanThreads = 1024;
constexpr int kProfThreads = 256;
constexpr int kFftThreads = 256;
constexpr int kTile = 4096;          // complex fp64 values per LDS tile (64 KiB)
constexpr int kTargetThreads = 1 << 18;

// carry-save adder on 32 bit positions at once: a + b + c = 2 h + l
__device__ __forceinline__ void csa(uint32_t &h, uint32_t &l, uint32_t a, uint32_t b, uint32_t c)
{
    const uint32_t u = a ^ b;
    h = (a & b) | (u & c);
    l = u ^ c;
}

// Column popcount of the sigma_x plane.  Thread (chunk, word column wc)
// counts bit by bit over rows [chunk R, chunk R + R) with bit-sliced
// counters: ones/twos/fours/eights hold the count modulo 16 of each of the
// 32 columns, every 16 rows the carry out ("sixteens") goes into byte-lane
// counters, which spill into 16-bit lanes every 255 groups.  Writes
// partial[chunk * Lx + 32 wc + b] in stored-column order.
__global__ __launch_bounds__(kCountThreads) void colcount_kernel(const uint32_t *plane, int32_t Ly,
                                                                 int32_t W, int32_t R, int32_t nch,
                                                                 int32_t *partial)
{
    const int64_t t = (int64_t)blockIdx.x * kCountThreads + threadIdx.x;
    if (t >= (int64_t)W * nch) return;
    const int wc = (int)(t % W), ch = (int)(t / W);
    const int y0 = ch * R, y1 = min(Ly, y0 + R);
    const uint32_t *col = plane + wc;

    uint32_t ones = 0, twos = 0, fours = 0, eights = 0;
    uint32_t acc[8], lo[8], hi[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = lo[j] = hi[j] = 0u;
    auto spill = [&]() {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            lo[j] += acc[j] & 0x00FF00FFu;
            hi[j] += (acc[j] >> 8) & 0x00FF00FFu;
            acc[j] = 0u;
        }
    };
    int groups = 0;
    for (int y = y0; y < y1; y += 16) {
        uint32_t w[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) w[i] = (y + i < y1) ? col[(size_t)(y + i) * W] : 0u;
        uint32_t twosA, twosB, foursA, foursB, eightsA, eightsB, sixteens;
        csa(twosA, ones, ones, w[0], w[1]);
        csa(twosB, ones, ones, w[2], w[3]);
        csa(foursA, twos, twos, twosA, twosB);
        csa(twosA, ones, ones, w[4], w[5]);
        csa(twosB, ones, ones, w[6], w[7]);
        csa(foursB, twos, twos, twosA, twosB);
        csa(eightsA, fours, fours, foursA, foursB);
        csa(twosA, ones, ones, w[8], w[9]);
        csa(twosB, ones, ones, w[10], w[11]);
        csa(foursA, twos, twos, twosA, twosB);
        csa(twosA, ones, ones, w[12], w[13]);
        csa(twosB, ones, ones, w[14], w[15]);
        csa(foursB, twos, twos, twosA, twosB);
        csa(eightsB, fours, fours, foursA, foursB);
        csa(sixteens, eights, eights, eightsA, eightsB);
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += (sixteens >> j) & 0x01010101u;
        if (++groups == 255) {
            spill();
            groups = 0;
        }
    }
    spill();
    int32_t c[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        const int j = b & 7, m = b >> 3;
        const uint32_t lane16 = (((m & 1) ? hi[j] : lo[j]) >> (16 * (m >> 1))) & 0xffffu;
        c[b] = (int32_t)(16 * lane16 + 8 * ((eights >> b) & 1u) + 4 * ((fours >> b) & 1u) +
                         2 * ((twos >> b) & 1u) + ((ones >> b) & 1u));
    }
    int4 *out = reinterpret_cast<int4 *>(partial + (size_t)ch * 32 * W + 32 * (size_t)wc);
#pragma unroll
    for (int v = 0; v < 8; ++v) out[v] = make_int4(c[4 * v], c[4 * v + 1], c[4 * v + 2], c[4 * v + 3]);
}

__global__ void colsum_kernel(const int32_t *partial, int32_t nch, int32_t Lx, int32_t *cnt)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Lx) return;
    int32_t s = 0;
    for (int ch = 0; ch < nch; ++ch) s += partial[(size_t)ch * Lx + c];
    cnt[c] = s;
}

// The profiles as scans of integer steps d(i):
//   v(i) = scale * sum_{i'<i} d(i') + e(i),
// column profile X: d(l) = 2 c(stored column of l) - Ly, scale 1, e = 0;
// row profile Y: d(y) = 2 sigma_y-bit(0,y) - 1, scale Lx, e(y) = the row's
// sum of P.  Every v is an integer below 2^41 in magnitude, exact in fp64.
// Three launches over blocks of kProfThreads values: block sums of d and of
// v's contributions (sum_i v(i) = scale sum_j d(j) (n-1-j) + sum_j e(j)); one
// workgroup scans the block sums and forms the mean; every block rescans its
// values and writes v(i) - mean into the real parts of z.
template <bool kRows>
__device__ __forceinline__ int64_t profile_step(const int32_t *cnt, const int64_t *rows, int32_t Lx,
                                                int32_t Ly, int32_t ox, int i)
{
    if (kRows) return 2 * rows[2 * (size_t)Ly + i] - 1;
    int xs = i - ox;
    if (xs < 0) xs += Lx;
    return 2 * (int64_t)cnt[xs] - Ly;
}

// blk[2 b] = sum of d over block b, blk[2 b + 1] = its part of sum_i v(i).
template <bool kRows>
__global__ __launch_bounds__(kProfThreads) void profile_sums_kernel(const int32_t *cnt,
                                                                    const int64_t *rows, int32_t Lx,
                                                                    int32_t Ly, int32_t ox,
                                                                    int64_t *blk)
{
    __shared__ int64_t lds[32];
    const int n = kRows ? Ly : Lx;
    const int64_t scale = kRows ? (int64_t)Lx : 1;
    const int i = blockIdx.x * kProfThreads + threadIdx.x;
    const int64_t d = i < n ? profile_step<kRows>(cnt, rows, Lx, Ly, ox, i) : 0;
    const int64_t e = (kRows && i < n) ? rows[i] : 0;
    const int64_t w = i < n ? scale * d * (int64_t)(n - 1 - i) + e : 0;
    const __int128 D = core::block_sum_i128(d, lds);
    const __int128 V = core::block_sum_i128(w, lds);
    if (threadIdx.x == 0) {
        blk[2 * (size_t)blockIdx.x] = (int64_t)D;
        blk[2 * (size_t)blockIdx.x + 1] = (int64_t)V;
    }
}

// In place: blk[2 b] becomes the exclusive prefix of the block sums of d;
// blk[2 nb] receives the mean of v as the bits of a double.
__global__ __launch_bounds__(kScanThreads) void profile_offsets_kernel(int64_t *blk, int32_t nb,
                                                                       int32_t n)
{
    __shared__ int64_t lds[32];
    const int per = (nb + kScanThreads - 1) / kScanThreads;
    const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
    int64_t local = 0, vs = 0;
    for (int b = b0; b < b1; ++b) {
        local += blk[2 * (size_t)b];
        vs += blk[2 * (size_t)b + 1];
    }
    int64_t unused;
    int64_t run = core::block_exclusive_scan(local, lds, &unused);
    const __int128 V = core::block_sum_i128(vs, lds);
    for (int b = b0; b < b1; ++b) {
        const int64_t d = blk[2 * (size_t)b];
        blk[2 * (size_t)b] = run;
        run += d;
    }
    if (threadIdx.x == 0) {
        const double mean = (double)(int64_t)V / n;  // its rounding only moves n = 0
        blk[2 * (size_t)nb] = __double_as_longlong(mean);
    }
}

template <bool kRows>
__global__ __launch_bounds__(kProfThreads) void profile_write_kernel(const int32_t *cnt,
                                                                     const int64_t *rows,
                                                                     int32_t Lx, int32_t Ly,
                                                                     int32_t ox, const int64_t *blk,
                                                                     int32_t nb, double2 *z)
{
    __shared__ int64_t lds[16];
    const int n = kRows ? Ly : Lx;
    const int64_t scale = kRows ? (int64_t)Lx : 1;
    const int i = blockIdx.x * kProfThreads + threadIdx.x;
    const int64_t d = i < n ? profile_step<kRows>(cnt, rows, Lx, Ly, ox, i) : 0;
    int64_t unused;
    const int64_t pre = blk[2 * (size_t)blockIdx.x] + core::block_exclusive_scan(d, lds, &unused);
    if (i >= n) return;
    const int64_t v = scale * pre + (kRows ? rows[i] : 0);
    const double mean = __longlong_as_double(blk[2 * (size_t)nb]);
    z[i] = make_double2((double)v - mean, 0.0);
}

// z <- (z + w) at i, (z - w) e^{-i pi (i mod 2h) / h} at i + h: one radix-2
// decimation-in-frequency stage of span h on blocks of 2h values.
__device__ __forceinline__ void dif_butterfly(double2 &a, double2 &b, int r, int h)
{
    double s, c;
    sincospi(-(double)r / h, &s, &c);
    const double2 u = a, v = b;
    a = make_double2(u.x + v.x, u.y + v.y);
    const double dx = u.x - v.x, dy = u.y - v.y;
    b = make_double2(dx * c - dy * s, dx * s + dy * c);
}

__global__ __launch_bounds__(kFftThreads) void fft_stage_kernel(double2 *z, int32_t n, int32_t h)
{
    const int i = blockIdx.x * kFftThreads + threadIdx.x;  // butterfly index
    if (i >= (n >> 1)) return;
    const int r = i & (h - 1);
    const int lo = ((i - r) << 1) + r;
    double2 a = z[lo], b = z[lo + h];
    dif_butterfly(a, b, r, h);
    z[lo] = a;
    z[lo + h] = b;
}

// The remaining stages (spans T/2 .. 1) of one contiguous tile of T values
// in LDS.
__global__ __launch_bounds__(kFftThreads) void fft_tile_kernel(double2 *z, int32_t T)
{
    __shared__ double2 tile[kTile];
    double2 *g = z + (size_t)blockIdx.x * T;
    for (int i = threadIdx.x; i < T; i += kFftThreads) tile[i] = g[i];
    __syncthreads();
    for (int h = T >> 1; h >= 1; h >>= 1) {
        for (int i = threadIdx.x; i < (T >> 1); i += kFftThreads) {
            const int r = i & (h - 1);
            const int lo = ((i - r) << 1) + r;
            double2 a = tile[lo], b = tile[lo + h];
            dif_butterfly(a, b, r, h);
            tile[lo] = a;
            tile[lo + h] = b;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < T; i += kFftThreads) g[i] = tile[i];
}

// S(n) = |Z(n)|^2 / (Lx Ly) for n = 0 .. len/2 from the bit-reversed
// transform; S(0) = 0 exactly (the mean is subtracted by definition).
__global__ void spectrum_kernel(const double2 *z, int32_t len, int32_t log2len, double norm,
                                double *S)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > (len >> 1)) return;
    const uint32_t j = __brev((uint32_t)k) >> (32 - log2len);
    const double2 v = z[j];
    S[k] = k == 0 ? 0.0 : (v.x * v.x + v.y * v.y) * norm;
}

int log2_exact(int32_t n)
{
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}

hipError_t launch_fft(double2 *z, int32_t n, hipStream_t st)
{
    const int T = n < kTile ? n : kTile;
    for (int32_t h = n >> 1; 2 * h > T; h >>= 1)
        hipLaunchKernelGGL(fft_stage_kernel, dim3((n / 2 + kFftThreads - 1) / kFftThreads),
                           dim3(kFftThreads), 0, st, z, n, h);
    hipLaunchKernelGGL(fft_tile_kernel, dim3(n / T), dim3(kFftThreads), 0, st, z, T);
    return hipGetLastError();
}

}  // namespace

bool psd_shape_ok(int64_t Lx, int64_t Ly)
{
    auto pow2 = [](int64_t v) { return v > 0 && (v & (v - 1)) == 0; };
    return pow2(Lx) && pow2(Ly);
}

PsdPlan psd_plan(int64_t Lx, int64_t Ly)
{
    PsdPlan p{};
    const int64_t W = Lx / 32;
    const int64_t want = (kTargetThreads + W - 1) / W;  // chunks for ~2^18 threads
    int64_t R = (Ly + want - 1) / want;
    R = (R + 15) / 16 * 16;
    p.R = (int32_t)R;
    p.nch = (int32_t)((Ly + R - 1) / R);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    p.off_cnt = al((size_t)p.nch * Lx * 4);
    p.off_zx = p.off_cnt + al((size_t)Lx * 4);
    p.off_zy = p.off_zx + al((size_t)Lx * 16);
    p.off_spec = p.off_zy + al((size_t)Ly * 16);
    p.off_blk = p.off_spec + al((size_t)(Lx / 2 + 1 + Ly / 2 + 1) * 8);
    const size_t nbx = (Lx + kProfThreads - 1) / kProfThreads, nby = (Ly + kProfThreads - 1) / kProfThreads;
    p.bytes = p.off_blk + al((2 * (nbx + nby) + 4) * 8);
    return p;
}

hipError_t launch_psd(const LatticeView &v, const PsdPlan &p, const int64_t *rows, void *scratch,
                      hipStream_t st)
{
    char *base = static_cast<char *>(scratch);
    int32_t *partial = reinterpret_cast<int32_t *>(base);
    int32_t *cnt = reinterpret_cast<int32_t *>(base + p.off_cnt);
    double2 *zx = reinterpret_cast<double2 *>(base + p.off_zx);
    double2 *zy = reinterpret_cast<double2 *>(base + p.off_zy);
    double *spec = reinterpret_cast<double *>(base + p.off_spec);

    const int64_t nthr = (int64_t)v.W * p.nch;
    hipLaunchKernelGGL(colcount_kernel, dim3((unsigned)((nthr + kCountThreads - 1) / kCountThreads)),
                       dim3(kCountThreads), 0, st, v.planes, v.Ly, v.W, p.R, p.nch, partial);
    hipLaunchKernelGGL(colsum_kernel, dim3((v.Lx + 255) / 256), dim3(256), 0, st, partial, p.nch,
                       v.Lx, cnt);
    const int32_t nbx = (v.Lx + kProfThreads - 1) / kProfThreads;
    const int32_t nby = (v.Ly + kProfThreads - 1) / kProfThreads;
    int64_t *bx = reinterpret_cast<int64_t *>(base + p.off_blk);
    int64_t *by = bx + 2 * (size_t)nbx + 2;
    hipLaunchKernelGGL(profile_sums_kernel<false>, dim3(nbx), dim3(kProfThreads), 0, st, cnt, rows,
                       v.Lx, v.Ly, v.ox, bx);
    hipLaunchKernelGGL(profile_sums_kernel<true>, dim3(nby), dim3(kProfThreads), 0, st, cnt, rows,
                       v.Lx, v.Ly, v.ox, by);
    hipLaunchKernelGGL(profile_offsets_kernel, dim3(1), dim3(kScanThreads), 0, st, bx, nbx, v.Lx);
    hipLaunchKernelGGL(profile_offsets_kernel, dim3(1), dim3(kScanThreads), 0, st, by, nby, v.Ly);
    hipLaunchKernelGGL(profile_write_kernel<false>, dim3(nbx), dim3(kProfThreads), 0, st, cnt, rows,
                       v.Lx, v.Ly, v.ox, bx, nbx, zx);
    hipLaunchKernelGGL(profile_write_kernel<true>, dim3(nby), dim3(kProfThreads), 0, st, cnt, rows,
                       v.Lx, v.Ly, v.ox, by, nby, zy);
    hipError_t e = launch_fft(zx, v.Lx, st);
    if (e != hipSuccess) return e;
    e = launch_fft(zy, v.Ly, st);
    if (e != hipSuccess) return e;
    const double norm = 1.0 / ((double)v.Lx * (double)v.Ly);
    hipLaunchKernelGGL(spectrum_kernel, dim3((v.Lx / 2 + 256) / 256), dim3(256), 0, st, zx, v.Lx,
                       log2_exact(v.Lx), norm, spec);
    hipLaunchKernelGGL(spectrum_kernel, dim3((v.Ly / 2 + 256) / 256), dim3(256), 0, st, zy, v.Ly,
                       log2_exact(v.Ly), norm, spec + v.Lx / 2 + 1);
    return hipGetLastError();
}

}  // namespace okpz
