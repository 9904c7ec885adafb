// Device side of the exact squared width (Sec. I height reconstruction,
// Eq. (Wdef)); shared by the per-lattice width kernels and the persistent
// batch kernel.
//
// h(x,y) = H0 + G(y) + P_y(x), with G(y) = sum_{k<y} sigma_y(0,k) and
// P_y(x) = sum_{l<x} sigma_x(l,y).  width_row: one wavefront reads row y's
// words once, in stored order with aligned 16-byte loads; each lane takes
// four consecutive words, sums them chunk by chunk through a 256-entry table
// of 8-site partial sums, a wavefront prefix scan of the segments' height
// changes gives every segment's starting height, and the row's rotation is
// undone in closed form at the end.  width_combine: one workgroup
// scans the column-0 sigma_y bits to get G(y) and combines the rows into
// 128-bit S1' = sum (h - H0) and S2' = sum (h - H0)^2.
#pragma once

#include "okpz_internal.h"

namespace okpz {
namespace core {

// Table of 8-site chunks.  For a byte c (bit i = site i, sigma_i = +1 when
// set) and the partial heights q_0 = 0, q_{i+1} = q_i + sigma_i, entry c holds
// s2 = sum_{i<8} q_i^2 in bits 0..7, s1 = sum_{i<8} q_i in bits 8..15 and
// d = q_8 in bits 16..23 (s1 and d as signed bytes).  A chunk whose first site
// sits at height B then adds 8 B + s1 to the sum of heights and
// 8 B^2 + 2 B s1 + s2 to the sum of squares.  Built by the whole workgroup;
// the caller synchronises before use.
__device__ __forceinline__ void width_lut_build(uint32_t *lut)
{
    for (int c = threadIdx.x; c < 256; c += blockDim.x) {
        int32_t q = 0, s1 = 0, s2 = 0;
        for (int i = 0; i < 8; ++i) {
            s1 += q;
            s2 += q * q;
            q += ((c >> i) & 1) ? 1 : -1;
        }
        lut[c] = (uint32_t)s2 | ((uint32_t)(s1 & 0xff) << 8) | ((uint32_t)(q & 0xff) << 16);
    }
}

// Row y of lattice view v by one wavefront (lane = threadIdx.x & 63); lane 0
// writes rows[y] = sum_x P, rows[Ly + y] = sum_x P^2, rows[2 Ly + y] = the
// sigma_y bit at physical column 0.  lut: the chunk table in LDS.
//
// The row is read in stored order, kWpl words per lane per pass (four: one
// aligned 16-byte load; one for narrow rows, with fewer registers).
// With Q(c) the sigma_x prefix over stored columns c' < c and xs0 the stored
// column of physical column 0, the full row sums to zero (a periodic row), so
// P(x) = Q((xs0 + x) mod Lx) - Q(xs0) for every x; the physical sums follow
// from the stored-order ones:
//   sum P = sum Q - Lx Q(xs0),  sum P^2 = sum Q^2 - 2 Q(xs0) sum Q + Lx Q(xs0)^2.
template <int kWpl = 4>
__device__ __forceinline__ void width_row(const LatticeView &v, int y, int lane,
                                         const uint32_t *lut, int64_t *rows)
{
    const uint32_t *row = v.planes + (size_t)y * v.W;
    const int xs0 = (v.Lx - v.ox) % v.Lx;  // stored column of physical column 0
    const int wq = xs0 >> 5;
    const uint32_t bq = (uint32_t)(xs0 & 31);
    const bool vec = (v.W & 3) == 0;  // rows are 16-byte aligned

    int64_t a1 = 0, a2 = 0, q0 = 0;
    int32_t carry = 0;
    for (int base = 0; base < v.W; base += 64 * kWpl) {
        const int k0 = base + lane * kWpl;
        const int nw = max(0, min(kWpl, v.W - k0));  // words of this lane
        uint32_t wd[kWpl];
#pragma unroll
        for (int t = 0; t < kWpl; ++t) wd[t] = 0u;
        if (kWpl == 4 && vec && nw == kWpl) {
            const uint4 q = *reinterpret_cast<const uint4 *>(row + k0);
            wd[0] = q.x; wd[1] = q.y; wd[2] = q.z; wd[3] = q.w;
        } else {
#pragma unroll
            for (int t = 0; t < kWpl; ++t)
                if (t < nw) wd[t] = row[k0 + t];
        }
        // heights relative to the first site of the lane's segment; every
        // pass but the last has four words in every lane (a uniform test)
        int32_t B = 0, S1 = 0, S2 = 0;
        auto chunks = [&](uint32_t word) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t e = lut[(word >> (8 * j)) & 255u];
                const int32_t s2 = (int32_t)(e & 0xffu);
                const int32_t s1 = (int32_t)(int8_t)(e >> 8);
                const int32_t d = (int32_t)(int8_t)(e >> 16);
                const int32_t t1 = 8 * B + s1;
                S1 += t1;
                S2 += __mul24(B, t1 + s1) + s2;  // |B| <= 128: a 24-bit multiply
                B += d;
            }
        };
        if (base + 64 * kWpl <= v.W) {
#pragma unroll
            for (int t = 0; t < kWpl; ++t) chunks(wd[t]);
        } else {
#pragma unroll
            for (int t = 0; t < kWpl; ++t)
                if (t < nw) chunks(wd[t]);
        }
        // Q(xs0): only in the pass holding word wq (a uniform test), and there
        // only in the lane holding it
        int32_t qrel = 0;
        bool hasq = false;
        if (wq >= base && wq < base + 64 * kWpl) {
            const int tq = wq - k0;
            if (tq >= 0 && tq < kWpl) {
                int32_t Bq = 0;
                uint32_t word = wd[0];
#pragma unroll
                for (int t = 1; t < kWpl; ++t) {
                    if (t <= tq) {
                        Bq += 2 * (int32_t)__popc(wd[t - 1]) - 32;
                        word = wd[t];
                    }
                }
                const uint32_t below = bq ? (word & ((1u << bq) - 1u)) : 0u;
                qrel = Bq + 2 * (int32_t)__popc(below) - (int32_t)bq;
                hasq = true;
            }
        }
        int32_t incl = B;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        const int64_t b = carry + incl - B;  // Q at the segment's first site
        const int64_t n = 32 * nw;
        a1 += n * b + S1;
        a2 += n * b * b + 2 * b * S1 + S2;
        if (hasq) q0 = b + qrel;
        carry += __shfl(incl, 63, 64);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a1 += __shfl_down(a1, o, 64);
        a2 += __shfl_down(a2, o, 64);
        q0 += __shfl_down(q0, o, 64);  // one lane holds Q(xs0)
    }
    if (lane == 0) {
        const int64_t L = v.Lx;
        const uint32_t *rowy = v.planes + ((size_t)v.Ly + y) * v.W;
        const uint32_t cb = (rowy[wq] >> bq) & 1u;
        rows[y] = a1 - L * q0;
        rows[(size_t)v.Ly + y] = a2 - 2 * q0 * a1 + L * q0 * q0;
        rows[2 * (size_t)v.Ly + y] = (int64_t)cb;
    }
}

// Exclusive prefix sum of v over the workgroup in thread order; *total gets
// the workgroup's sum.  lds: 16 entries.  Ends with a barrier.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *lds, int64_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    int64_t off = 0, tot = 0;
    for (int w = 0; w < nwave; ++w) {
        const int64_t s = lds[w];
        if (w < wave) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// Sum of a 128-bit value over the workgroup, returned in every thread.
// lds: 32 entries.  Ends with a barrier.
__device__ __forceinline__ __int128 block_sum_i128(__int128 v, int64_t *lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    uint64_t lo = (uint64_t)v, hi = (uint64_t)((unsigned __int128)v >> 64);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t alo = __shfl_down(lo, o, 64), ahi = __shfl_down(hi, o, 64);
        const unsigned __int128 s = (((unsigned __int128)hi << 64) | lo) +
                                    (((unsigned __int128)ahi << 64) | alo);
        lo = (uint64_t)s;
        hi = (uint64_t)(s >> 64);
    }
    if (lane == 0) {
        lds[2 * wave] = (int64_t)lo;
        lds[2 * wave + 1] = (int64_t)hi;
    }
    __syncthreads();
    unsigned __int128 t = 0;
    for (int w = 0; w < nwave; ++w)
        t += ((unsigned __int128)(uint64_t)lds[2 * w + 1] << 64) | (uint64_t)lds[2 * w];
    __syncthreads();
    return (__int128)t;
}

// Combine the rows into out[0..3] = {S1' lo, S1' hi, S2' lo, S2' hi} (128-bit
// two's complement halves) with one workgroup of up to 1024 threads.  Each
// thread takes a run of rows; the column-0 prefix G(y) comes from a
// wavefront scan plus the totals of the lower waves; sums of squares are
// accumulated in 128 bits and reduced wave by wave.  lds: 64 entries of LDS
// scratch.  Ends with a barrier.
__device__ __forceinline__ void width_combine(const int64_t *rows, int32_t Lx, int32_t Ly,
                                              int64_t *out, int64_t *lds)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwave = nth >> 6;
    const int per = (Ly + nth - 1) / nth;
    const int ya = min(Ly, tid * per), yb = min(Ly, ya + per);
    const int64_t *rs1 = rows, *rs2 = rows + Ly, *col = rows + 2 * (size_t)Ly;

    int32_t local = 0;
    for (int y = ya; y < yb; ++y) local += 2 * (int32_t)col[y] - 1;
    int32_t incl = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    int64_t G = incl - local;  // sum of sigma_y(0,k) for k < ya
    for (int w = 0; w < wave; ++w) G += lds[w];

    int64_t s1 = 0;
    __int128 s2 = 0;
    for (int y = ya; y < yb; ++y) {
        const int64_t p1 = rs1[y], p2 = rs2[y];
        s1 += (int64_t)Lx * G + p1;
        s2 += (__int128)((int64_t)Lx * G * G + 2 * G * p1 + p2);
        G += 2 * col[y] - 1;
    }
    uint64_t lo = (uint64_t)s2;
    uint64_t hi = (uint64_t)(s2 >> 64);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t a1 = __shfl_down(s1, o, 64);
        const uint64_t alo = __shfl_down(lo, o, 64);
        const uint64_t ahi = __shfl_down(hi, o, 64);
        s1 += a1;
        const unsigned __int128 v = (((unsigned __int128)hi << 64) | lo) +
                                    (((unsigned __int128)ahi << 64) | alo);
        lo = (uint64_t)v;
        hi = (uint64_t)(v >> 64);
    }
    __syncthreads();  // the scan totals are read above; lds is reused
    if (lane == 0) {
        lds[16 + wave] = s1;
        lds[32 + wave] = (int64_t)lo;
        lds[48 + wave] = (int64_t)hi;
    }
    __syncthreads();
    if (tid == 0) {
        __int128 t1 = 0;
        unsigned __int128 t2 = 0;
        for (int w = 0; w < nwave; ++w) {
            t1 += lds[16 + w];
            t2 += ((unsigned __int128)(uint64_t)lds[48 + w] << 64) | (uint64_t)lds[32 + w];
        }
        out[0] = (int64_t)(uint64_t)t1;
        out[1] = (int64_t)(t1 >> 64);
        out[2] = (int64_t)(uint64_t)t2;
        out[3] = (int64_t)(uint64_t)(t2 >> 64);
    }
    __syncthreads();
}

}  // namespace core
}  // namespace okpz
