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
// A side that is not a power of two goes through Bluestein's chirp-z form
// (Bluestein 1970): with c_j = exp(-i pi j^2 / n), X_k = c_k sum_j (x_j c_j)
// conj(c_{k-j}), a convolution done with power-of-two transforms of length
// M >= 2n - 1 (forward stages, a pointwise product in bit-reversed order, and
// the forward stages undone in reverse order, which returns natural order).
#include "psd.h"
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

// The stage above undone without its factor 1/2: (a, b) <- (a + t, a - t),
// t = b e^{+i pi r / h}.  All stages undone in reverse order turn the
// bit-reversed transform of x back into n x in natural order, i.e. they
// apply the unnormalised inverse DFT to a bit-reversed spectrum.
__device__ __forceinline__ void dif_butterfly_undo(double2 &a, double2 &b, int r, int h)
{
    double s, c;
    sincospi((double)r / h, &s, &c);
    const double2 t = make_double2(b.x * c - b.y * s, b.x * s + b.y * c);
    const double2 u = a;
    a = make_double2(u.x + t.x, u.y + t.y);
    b = make_double2(u.x - t.x, u.y - t.y);
}

template <bool kUndo>
__global__ __launch_bounds__(kFftThreads) void fft_stage_kernel(double2 *z, int32_t n, int32_t h)
{
    const int i = blockIdx.x * kFftThreads + threadIdx.x;  // butterfly index
    if (i >= (n >> 1)) return;
    const int r = i & (h - 1);
    const int lo = ((i - r) << 1) + r;
    double2 a = z[lo], b = z[lo + h];
    if (kUndo)
        dif_butterfly_undo(a, b, r, h);
    else
        dif_butterfly(a, b, r, h);
    z[lo] = a;
    z[lo + h] = b;
}

// The stages of spans T/2 .. 1 (undone: 1 .. T/2) of one contiguous tile of
// T values, in LDS.
template <bool kUndo>
__global__ __launch_bounds__(kFftThreads) void fft_tile_kernel(double2 *z, int32_t T)
{
    __shared__ double2 tile[kTile];
    double2 *g = z + (size_t)blockIdx.x * T;
    for (int i = threadIdx.x; i < T; i += kFftThreads) tile[i] = g[i];
    __syncthreads();
    for (int k = 0; (1 << k) < T; ++k) {
        const int h = kUndo ? (1 << k) : (T >> (k + 1));
        for (int i = threadIdx.x; i < (T >> 1); i += kFftThreads) {
            const int r = i & (h - 1);
            const int lo = ((i - r) << 1) + r;
            double2 a = tile[lo], b = tile[lo + h];
            if (kUndo)
                dif_butterfly_undo(a, b, r, h);
            else
                dif_butterfly(a, b, r, h);
            tile[lo] = a;
            tile[lo + h] = b;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < T; i += kFftThreads) g[i] = tile[i];
}

// c_j = exp(-i pi j^2 / n), the phase reduced exactly: j^2 mod 2n.
__device__ __forceinline__ double2 chirp(int64_t j, int32_t n)
{
    const int64_t k = (j * j) % (2 * (int64_t)n);
    double s, c;
    sincospi(-(double)k / n, &s, &c);
    return make_double2(c, s);
}

// A = (x_j c_j, then zeros) and B = (conj(c_m) at m and M - m for m < n,
// zeros between), both of length M.
__global__ void chirp_kernel(const double2 *x, int32_t n, int32_t M, double2 *A, double2 *B)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    if (j < n) {
        const double2 c = chirp(j, n), v = x[j];
        A[j] = make_double2(v.x * c.x - v.y * c.y, v.x * c.y + v.y * c.x);
    } else {
        A[j] = make_double2(0.0, 0.0);
    }
    const int m = j < n ? j : (j > M - n ? M - j : -1);
    if (m >= 0) {
        const double2 c = chirp(m, n);
        B[j] = make_double2(c.x, -c.y);
    } else {
        B[j] = make_double2(0.0, 0.0);
    }
}

__global__ void cmul_kernel(double2 *A, const double2 *B, int32_t M)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double2 a = A[j], b = B[j];
    A[j] = make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// X_k = c_k conv_k, conv = (the undone transform) / M, natural order.
__global__ void unchirp_kernel(const double2 *conv, int32_t n, int32_t M, double2 *x)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double2 c = chirp(k, n), v = conv[k];
    const double inv = 1.0 / M;
    x[k] = make_double2((v.x * c.x - v.y * c.y) * inv, (v.x * c.y + v.y * c.x) * inv);
}

// S(n) = |Z(n)|^2 / (Lx Ly) for n = 0 .. len/2 from the transform, in
// bit-reversed order (log2len > 0) or natural order (log2len = 0); S(0) = 0
// exactly (the mean is subtracted by definition).
__global__ void spectrum_kernel(const double2 *z, int32_t len, int32_t log2len, double norm,
                                double *S)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > (len >> 1)) return;
    const uint32_t j = log2len > 0 ? __brev((uint32_t)k) >> (32 - log2len) : (uint32_t)k;
    const double2 v = z[j];
    S[k] = k == 0 ? 0.0 : (v.x * v.x + v.y * v.y) * norm;
}

int log2_exact(int32_t n)
{
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Bluestein length for a side n: the power of two M >= 2n - 1.
int64_t conv_len(int64_t n)
{
    int64_t M = 1;
    while (M < 2 * n - 1) M <<= 1;
    return M;
}

// Forward transform of n = 2^k values in place, output bit-reversed.
hipError_t launch_fft(double2 *z, int32_t n, hipStream_t st)
{
    const int T = n < kTile ? n : kTile;
    for (int32_t h = n >> 1; 2 * h > T; h >>= 1)
        hipLaunchKernelGGL(fft_stage_kernel<false>, dim3((n / 2 + kFftThreads - 1) / kFftThreads),
                           dim3(kFftThreads), 0, st, z, n, h);
    hipLaunchKernelGGL(fft_tile_kernel<false>, dim3(n / T), dim3(kFftThreads), 0, st, z, T);
    return hipGetLastError();
}

// launch_fft undone: bit-reversed spectrum in, n x the inverse DFT out.
hipError_t launch_fft_undo(double2 *z, int32_t n, hipStream_t st)
{
    const int T = n < kTile ? n : kTile;
    hipLaunchKernelGGL(fft_tile_kernel<true>, dim3(n / T), dim3(kFftThreads), 0, st, z, T);
    for (int32_t h = T; h < n; h <<= 1)
        hipLaunchKernelGGL(fft_stage_kernel<true>, dim3((n / 2 + kFftThreads - 1) / kFftThreads),
                           dim3(kFftThreads), 0, st, z, n, h);
    return hipGetLastError();
}

// The DFT of the n values of z, in place: bit-reversed when n is a power of
// two (returns log2 n), natural order through Bluestein otherwise (returns 0);
// A and B hold conv_len(n) values each.
hipError_t transform(double2 *z, int32_t n, double2 *A, double2 *B, int *order, hipStream_t st)
{
    if (pow2(n)) {
        *order = log2_exact(n);
        return launch_fft(z, n, st);
    }
    *order = 0;
    const int32_t M = (int32_t)conv_len(n);
    hipLaunchKernelGGL(chirp_kernel, dim3((M + 255) / 256), dim3(256), 0, st, z, n, M, A, B);
    hipError_t e = launch_fft(A, M, st);
    if (e != hipSuccess) return e;
    e = launch_fft(B, M, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cmul_kernel, dim3((M + 255) / 256), dim3(256), 0, st, A, B, M);
    e = launch_fft_undo(A, M, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(unchirp_kernel, dim3((n + 255) / 256), dim3(256), 0, st, A, n, M, z);
    return hipGetLastError();
}

}  // namespace

namespace {

// Scratch layout for column-count chunks of R rows (R a multiple of 16).
PsdPlan plan_with_rows(int64_t Lx, int64_t Ly, int64_t R)
{
    PsdPlan p{};
    p.R = (int32_t)R;
    p.nch = (int32_t)((Ly + R - 1) / R);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    p.off_cnt = al((size_t)p.nch * Lx * 4);
    p.off_zx = p.off_cnt + al((size_t)Lx * 4);
    p.off_zy = p.off_zx + al((size_t)Lx * 16);
    p.off_spec = p.off_zy + al((size_t)Ly * 16);
    p.off_blk = p.off_spec + al((size_t)(Lx / 2 + 1 + Ly / 2 + 1) * 8);
    const size_t nbx = (Lx + kProfThreads - 1) / kProfThreads, nby = (Ly + kProfThreads - 1) / kProfThreads;
    p.off_conv = p.off_blk + al((2 * (nbx + nby) + 4) * 8);
    int64_t M = 0;  // Bluestein buffers, shared by the two sides in turn
    if (!pow2(Lx)) M = conv_len(Lx);
    if (!pow2(Ly) && conv_len(Ly) > M) M = conv_len(Ly);
    p.conv_len = M;
    p.bytes = p.off_conv + 2 * al((size_t)M * 16);
    return p;
}

}  // namespace

PsdPlan psd_plan(int64_t Lx, int64_t Ly)
{
    const int64_t W = Lx / 32;
    const int64_t want = (kTargetThreads + W - 1) / W;  // chunks for ~2^18 threads
    int64_t R = (Ly + want - 1) / want;
    R = (R + 15) / 16 * 16;
    return plan_with_rows(Lx, Ly, R);
}

PsdPlan psd_plan_capped(int64_t Lx, int64_t Ly, size_t max_bytes)
{
    PsdPlan p = psd_plan(Lx, Ly);
    // fewer, taller chunks until the partial counts fit; a chunk's count of
    // one column must stay below 2^20 (16-bit lanes of sixteens)
    int64_t R = p.R;
    while (p.bytes > max_bytes && R < Ly && 2 * R < (int64_t(1) << 20)) {
        R *= 2;
        p = plan_with_rows(Lx, Ly, R);
    }
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
    double2 *A = reinterpret_cast<double2 *>(base + p.off_conv);
    double2 *B = reinterpret_cast<double2 *>(base + p.off_conv + (p.bytes - p.off_conv) / 2);
    int ox_order = 0, oy_order = 0;
    hipError_t e = transform(zx, v.Lx, A, B, &ox_order, st);
    if (e != hipSuccess) return e;
    e = transform(zy, v.Ly, A, B, &oy_order, st);
    if (e != hipSuccess) return e;
    const double norm = 1.0 / ((double)v.Lx * (double)v.Ly);
    hipLaunchKernelGGL(spectrum_kernel, dim3((v.Lx / 2 + 256) / 256), dim3(256), 0, st, zx, v.Lx,
                       ox_order, norm, spec);
    hipLaunchKernelGGL(spectrum_kernel, dim3((v.Ly / 2 + 256) / 256), dim3(256), 0, st, zy, v.Ly,
                       oy_order, norm, spec + v.Lx / 2 + 1);
    return hipGetLastError();
}

}  // namespace okpz
