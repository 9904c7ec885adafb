// C ABI of the okpz library: handles, validation, stream order, exact int64
// width combination, lattice up/download and checkpoints.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "okpz.h"
#include "host_logic.h"
#include "okpz_internal.h"
#include "psd.h"
#include "width.h"

struct okpz_sim {
    int64_t Lx, Ly;
    int32_t W;
    okpz::Geometry g;
    double p, q;
    uint64_t seed;
    uint32_t k0, k1;
    uint64_t Tp, Tq;
    uint32_t *buf[2];
    int copies;  // 2: ping-pong copies; 1: one copy updated in place
    int cur;
    int32_t ox;
    int64_t t;
    int64_t *d_h0;
    int64_t *d_out;
    int64_t *d_rows;
    hipStream_t stream;
    bool own_stream;
    void *mem;
    bool own_mem;
    int threads;  // sweep workgroup size (execution mapping only)
    int32_t cell_borders;  // OKPZ_CELLS_DEAD or OKPZ_CELLS_DELAYED
    void *psd_mem;  // spectrum scratch, allocated by the first okpz_psd
    int device;     // device current at creation, whose static scratch okpz_psd_noalloc uses
};

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(OKPZ_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                    \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

size_t plane_bytes(int64_t Lx, int64_t Ly) { return 2 * (size_t)Ly * (size_t)(Lx / 32) * 4; }

bool size_ok(int64_t L) { return okpz::host::side_ok(L); }

bool prob_ok(double v) { return v >= 0.0 && v <= 1.0; }

__global__ void init_flat_kernel(uint32_t *planes, int32_t Ly, int32_t W, int64_t *h0)
{
    // h(x,y) = (x+y) mod 2: sigma_x = sigma_y = +1 exactly where x+y is even
    const size_t n = 2 * (size_t)Ly * W;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t y = (e / W) % Ly;
        planes[e] = (y & 1) ? 0xAAAAAAAAu : 0x55555555u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *h0 = 0;
}

__global__ void set_h0_kernel(int64_t *h0, int64_t v) { *h0 = v; }

size_t state_bytes(int64_t Lx, int64_t Ly, int copies)
{
    return copies * align_up(plane_bytes(Lx, Ly)) + 2 * kAlign +
           align_up(okpz::width_scratch_words(Ly) * sizeof(int64_t));
}

int alloc_state(okpz_sim *s, void *dev_buf, size_t bytes, void *stream)
{
    const size_t pb = align_up(plane_bytes(s->Lx, s->Ly));
    const size_t need = state_bytes(s->Lx, s->Ly, s->copies);
    if (dev_buf) {
        if (bytes < need)
            return fail(OKPZ_ENOMEM, "buffer of %zu bytes, %zu needed", bytes, need);
        if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign)
            return fail(OKPZ_EINVAL, "device buffer must be %zu-byte aligned", kAlign);
        s->mem = dev_buf;
        s->own_mem = false;
        s->stream = reinterpret_cast<hipStream_t>(stream);
        s->own_stream = false;
    } else {
        void *m = nullptr;
        hipError_t e = hipMalloc(&m, need);
        if (e != hipSuccess) return fail(OKPZ_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
        s->mem = m;
        s->own_mem = true;
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            (void)hipFree(m);
            s->mem = nullptr;
            return hip_fail(e, "hipStreamCreate");
        }
        s->own_stream = true;
    }
    char *base = static_cast<char *>(s->mem);
    const size_t cb = s->copies * pb;
    s->buf[0] = reinterpret_cast<uint32_t *>(base);
    s->buf[1] = s->copies == 2 ? reinterpret_cast<uint32_t *>(base + pb) : s->buf[0];
    s->d_h0 = reinterpret_cast<int64_t *>(base + cb);
    s->d_out = reinterpret_cast<int64_t *>(base + cb + kAlign);
    s->d_rows = reinterpret_cast<int64_t *>(base + cb + 2 * kAlign);
    return OKPZ_OK;
}

void release(okpz_sim *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->psd_mem) (void)hipFree(s->psd_mem);
    if (s->own_mem && s->mem) (void)hipFree(s->mem);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// Spectrum scratch of okpz_psd_noalloc: one array per device, held until the
// process ends, never allocated or freed by a call.  In host code `scratch`
// names a host-side stand-in, not device memory: kernels and copies get the
// device address that hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticPsdBytes = size_t(24) << 20;
constexpr int64_t kStaticPsdMaxSide = int64_t(1) << 17;
static __device__ __align__(256) unsigned char scratch[kStaticPsdBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices];     // device address of `scratch` per device
bool g_static_tried[kMaxDevices];
hipError_t g_static_err[kMaxDevices];

// Once per device, with that device current (called from make_sim, the
// library's set-up of every handle).
void static_scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_tried[dev]) return;
    g_static_tried[dev] = true;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_static_err[dev] = e;
    g_static_ptr[dev] = e == hipSuccess ? ptr : nullptr;
}

void *static_scratch(int dev, hipError_t *err)
{
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_static_mu);
    *err = g_static_tried[dev] ? g_static_err[dev] : hipErrorNotInitialized;
    return g_static_ptr[dev];
}

int make_sim(okpz_sim **out, int64_t Lx, int64_t Ly, double p, double q, uint64_t seed,
             void *dev_buf, size_t bytes, void *stream, int copies = 2)
{
    if (!out) return fail(OKPZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (!size_ok(Lx) || !size_ok(Ly))
        return fail(OKPZ_EINVAL, "lattice %lldx%lld: sides must be multiples of 32 in [32, 2^20]",
                    (long long)Lx, (long long)Ly);
    if (!prob_ok(p) || !prob_ok(q)) return fail(OKPZ_EINVAL, "p=%g q=%g must lie in [0,1]", p, q);
    okpz_sim *s = new (std::nothrow) okpz_sim();
    if (!s) return fail(OKPZ_ENOMEM, "host allocation failed");
    s->Lx = Lx;
    s->Ly = Ly;
    s->W = (int32_t)(Lx / 32);
    okpz::geometry_of(Lx, Ly, &s->g);
    s->p = p;
    s->q = q;
    s->seed = seed;
    s->k0 = (uint32_t)(seed & 0xffffffffu);
    s->k1 = (uint32_t)(seed >> 32);
    s->Tp = okpz::threshold_of(p);
    s->Tq = okpz::threshold_of(q);
    s->copies = copies;
    s->cur = 0;
    s->ox = 0;
    s->t = 0;
    s->threads = 1024;
    const hipError_t de = hipGetDevice(&s->device);
    if (de != hipSuccess) {
        delete s;
        return hip_fail(de, "hipGetDevice");
    }
    static_scratch_setup(s->device);
    int rc = alloc_state(s, dev_buf, bytes, stream);
    if (rc != OKPZ_OK) {
        delete s;
        return rc;
    }
    *out = s;
    return OKPZ_OK;
}

int launch_flat(okpz_sim *s)
{
    const size_t n = 2 * (size_t)s->Ly * s->W;
    const int threads = 256;
    const int blocks = (int)std::min<size_t>((n + threads - 1) / threads, 65536);
    hipLaunchKernelGGL(init_flat_kernel, dim3(blocks), dim3(threads), 0, s->stream, s->buf[0],
                       (int32_t)s->Ly, s->W, s->d_h0);
    HIP_TRY(hipGetLastError());
    s->cur = 0;
    s->ox = 0;
    s->t = 0;
    return OKPZ_OK;
}

// physical column x of stored copy with offset ox: stored column (x - ox) mod Lx
inline int64_t stored_col(int64_t x, int32_t ox, int64_t Lx) { return ((x - ox) % Lx + Lx) % Lx; }

int download_rows(okpz_sim *s, int64_t y0, int64_t n, std::vector<uint32_t> &pl0,
                  std::vector<uint32_t> &pl1)
{
    const size_t W = (size_t)s->W;
    pl0.resize(n * W);
    pl1.resize(n * W);
    HIP_TRY(hipStreamSynchronize(s->stream));
    int64_t done = 0;
    while (done < n) {
        const int64_t y = (y0 + done) % s->Ly;
        const int64_t run = std::min<int64_t>(n - done, s->Ly - y);
        const uint32_t *src0 = s->buf[s->cur] + (size_t)y * W;
        const uint32_t *src1 = s->buf[s->cur] + ((size_t)s->Ly + y) * W;
        HIP_TRY(hipMemcpy(pl0.data() + done * W, src0, run * W * 4, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(pl1.data() + done * W, src1, run * W * 4, hipMemcpyDeviceToHost));
        done += run;
    }
    return OKPZ_OK;
}

void unpack_rows(const okpz_sim *s, int64_t n, const std::vector<uint32_t> &pl0,
                 const std::vector<uint32_t> &pl1, uint8_t *host)
{
    const int64_t Lx = s->Lx;
    const size_t W = (size_t)s->W;
    for (int64_t r = 0; r < n; ++r)
        for (int64_t x = 0; x < Lx; ++x) {
            const int64_t c = stored_col(x, s->ox, Lx);
            const uint32_t bx = (pl0[r * W + (c >> 5)] >> (c & 31)) & 1u;
            const uint32_t by = (pl1[r * W + (c >> 5)] >> (c & 31)) & 1u;
            host[r * Lx + x] = (uint8_t)(bx | (by << 1));
        }
}

int upload_lattice(okpz_sim *s, const uint8_t *host)
{
    const size_t W = (size_t)s->W;
    std::vector<uint32_t> planes(2 * (size_t)s->Ly * W, 0u);
    for (int64_t y = 0; y < s->Ly; ++y)
        for (int64_t x = 0; x < s->Lx; ++x) {
            const uint8_t b = host[y * s->Lx + x];
            if (b & 1) planes[(size_t)y * W + (x >> 5)] |= 1u << (x & 31);
            if (b & 2) planes[((size_t)s->Ly + y) * W + (x >> 5)] |= 1u << (x & 31);
        }
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemcpy(s->buf[0], planes.data(), planes.size() * 4, hipMemcpyHostToDevice));
    s->cur = 0;
    s->ox = 0;
    return OKPZ_OK;
}

using okpz::host::CkptHeader;

}  // namespace

namespace okpz {

bool geometry_of(int64_t Lx, int64_t Ly, Geometry *g)
{
    auto side = [](int64_t L) {
        int64_t b = 1;
        while (b < 256 && L % (b * 2) == 0) b *= 2;
        return (int32_t)b;
    };
    g->Bx = side(Lx);
    g->By = side(Ly);
    g->C = std::min<int32_t>(8, std::min(g->Bx, g->By));
    return true;
}

uint64_t threshold_of(double prob)
{
    if (!(prob > 0.0)) return 0;
    if (prob >= 1.0) return uint64_t(1) << 32;
    const long long r = std::llround(std::ldexp(prob, 32));
    return (uint64_t)std::clamp<long long>(r, 0, 1LL << 32);
}

}  // namespace okpz

extern "C" {

int okpz_geometry(int64_t Lx, int64_t Ly, int32_t *Bx, int32_t *By, int32_t *C)
{
    if (!size_ok(Lx) || !size_ok(Ly))
        return fail(OKPZ_EINVAL, "lattice sides must be multiples of 32 in [32, 2^20]");
    okpz::Geometry g;
    okpz::geometry_of(Lx, Ly, &g);
    if (Bx) *Bx = g.Bx;
    if (By) *By = g.By;
    if (C) *C = g.C;
    return OKPZ_OK;
}

size_t okpz_required_bytes(int64_t Lx, int64_t Ly)
{
    if (!size_ok(Lx) || !size_ok(Ly)) return 0;
    return state_bytes(Lx, Ly, 2);
}

size_t okpz_required_bytes_in_place(int64_t Lx, int64_t Ly)
{
    if (!size_ok(Lx) || !size_ok(Ly)) return 0;
    return state_bytes(Lx, Ly, 1);
}

int okpz_init(okpz_sim **out, int64_t Lx, int64_t Ly, double p, double q, uint64_t seed)
{
    return okpz_init_on(out, Lx, Ly, p, q, seed, nullptr, 0, nullptr);
}

int okpz_init_on(okpz_sim **out, int64_t Lx, int64_t Ly, double p, double q, uint64_t seed,
                 void *dev_buf, size_t bytes, void *hip_stream)
{
    if (!out) return fail(OKPZ_EINVAL, "out is NULL");
    *out = nullptr;
    okpz_sim *s = nullptr;
    int rc = make_sim(&s, Lx, Ly, p, q, seed, dev_buf, bytes, hip_stream);
    if (rc != OKPZ_OK) return rc;
    rc = launch_flat(s);
    if (rc != OKPZ_OK) {
        release(s);
        return rc;
    }
    *out = s;
    return OKPZ_OK;
}

int okpz_init_in_place(okpz_sim **out, int64_t Lx, int64_t Ly, double p, double q, uint64_t seed,
                       void *dev_buf, size_t bytes, void *hip_stream)
{
    if (!out) return fail(OKPZ_EINVAL, "out is NULL");
    *out = nullptr;
    okpz_sim *s = nullptr;
    int rc = make_sim(&s, Lx, Ly, p, q, seed, dev_buf, bytes, hip_stream, 1);
    if (rc != OKPZ_OK) return rc;
    rc = launch_flat(s);
    if (rc != OKPZ_OK) {
        release(s);
        return rc;
    }
    *out = s;
    return OKPZ_OK;
}

int okpz_get_copies(const okpz_sim *s, int32_t *copies)
{
    if (!s || !copies) return fail(OKPZ_EINVAL, "null argument");
    *copies = s->copies;
    return OKPZ_OK;
}

int okpz_sweep(okpz_sim *s, int64_t n_mcs)
{
    if (!s) return fail(OKPZ_EINVAL, "null handle");
    if (n_mcs < 0) return fail(OKPZ_EINVAL, "n_mcs < 0");
    if (s->t + n_mcs > (int64_t(1) << 32))
        return fail(OKPZ_EINVAL, "sweep index would pass 2^32");
    okpz::SweepLaunch a{};
    a.h0 = s->d_h0;
    a.Lx = (int32_t)s->Lx;
    a.Ly = (int32_t)s->Ly;
    a.W = s->W;
    a.Bx = s->g.Bx;
    a.By = s->g.By;
    a.nbx = (int32_t)(s->Lx / s->g.Bx);
    a.nby = (int32_t)(s->Ly / s->g.By);
    a.k0 = s->k0;
    a.k1 = s->k1;
    a.Tp = s->Tp;
    a.Tq = s->Tq;
    const bool trivial = (s->Tp == 0 || s->Tp == (uint64_t(1) << 32)) &&
                         (s->Tq == 0 || s->Tq == (uint64_t(1) << 32));
    a.need_accept_draws = trivial ? 0 : 1;
    a.delayed_cells = s->cell_borders == OKPZ_CELLS_DELAYED ? 1 : 0;
    for (int64_t n = 0; n < n_mcs; ++n) {
        const uint32_t sw = (uint32_t)s->t;
        int32_t sx, sy;
        okpz::block_shift(s->k0, s->k1, sw, s->g, &sx, &sy);
        const int64_t x00 = (s->Lx - sx) % s->Lx, y00 = (s->Ly - sy) % s->Ly;
        a.blk00 = (int32_t)((y00 / s->g.By) * a.nbx + x00 / s->g.Bx);
        a.u00 = (int32_t)(x00 % s->g.Bx);
        a.v00 = (int32_t)(y00 % s->g.By);
        a.src = s->buf[s->cur];
        a.dst = s->buf[s->cur ^ (s->copies - 1)];
        a.ox_src = s->ox;
        a.in_place = s->copies == 1 ? 1 : 0;
        a.sx = sx;
        a.sy = sy;
        a.s = sw;
        HIP_TRY(okpz::launch_sweep(a, s->threads, s->stream));
        if (s->copies == 2) {  // the destination copy holds block column 0 at stored 0
            s->cur ^= 1;
            s->ox = sx;
        }
        s->t += 1;
    }
    return OKPZ_OK;
}

static int measure(okpz_sim *s, __int128 *S1r, __int128 *S2r, int64_t *H0)
{
    okpz::LatticeView v{s->buf[s->cur], (int32_t)s->Lx, (int32_t)s->Ly, s->W, s->ox};
    HIP_TRY(okpz::launch_width(v, s->d_rows, s->d_out, s->stream));
    int64_t host[5];
    HIP_TRY(hipMemcpyAsync(host, s->d_out, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(host + 4, s->d_h0, sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    *S1r = (__int128)(((unsigned __int128)(uint64_t)host[1] << 64) | (uint64_t)host[0]);
    *S2r = (__int128)(((unsigned __int128)(uint64_t)host[3] << 64) | (uint64_t)host[2]);
    *H0 = host[4];
    return OKPZ_OK;
}

int okpz_width(okpz_sim *s, int64_t t, int64_t *sum_h, int64_t *sum_h2)
{
    if (!s) return fail(OKPZ_EINVAL, "null handle");
    if (t < s->t) return fail(OKPZ_EINVAL, "t=%lld is before the current time %lld", (long long)t,
                              (long long)s->t);
    int rc = okpz_sweep(s, t - s->t);
    if (rc != OKPZ_OK) return rc;
    __int128 S1r, S2r;
    int64_t H0;
    rc = measure(s, &S1r, &S2r, &H0);
    if (rc != OKPZ_OK) return rc;
    // S1 = S1' + N H0, S2 = S2' + 2 H0 S1' + N H0^2, exact in 128 bits
    const __int128 N = (__int128)s->Lx * s->Ly;
    const __int128 S1 = S1r + N * H0;
    const __int128 S2 = S2r + 2 * (__int128)H0 * S1r + N * (__int128)H0 * H0;
    const __int128 lim = (__int128)1 << 63;
    if (S1 >= lim || S1 < -lim || S2 >= lim || S2 < 0)
        return fail(OKPZ_EOVERFLOW, "width sums exceed int64 at t=%lld", (long long)s->t);
    if (sum_h) *sum_h = (int64_t)S1;
    if (sum_h2) *sum_h2 = (int64_t)S2;
    return OKPZ_OK;
}

int okpz_w2(okpz_sim *s, double *w2)
{
    if (!s || !w2) return fail(OKPZ_EINVAL, "null argument");
    __int128 S1r, S2r;
    int64_t H0;
    int rc = measure(s, &S1r, &S2r, &H0);
    if (rc != OKPZ_OK) return rc;
    const __int128 N = (__int128)s->Lx * s->Ly;
    const __int128 num = N * S2r - S1r * S1r;  // independent of H0
    *w2 = (double)num / ((double)N * (double)N);
    return OKPZ_OK;
}

int okpz_psd(okpz_sim *s, double *sx, double *sy)
{
    if (!s) return fail(OKPZ_EINVAL, "null handle");
    const okpz::PsdPlan p = okpz::psd_plan(s->Lx, s->Ly);
    if (!s->psd_mem) {
        hipError_t e = hipMalloc(&s->psd_mem, p.bytes);
        if (e != hipSuccess) {
            s->psd_mem = nullptr;
            return fail(OKPZ_ENOMEM, "hipMalloc(%zu): %s", p.bytes, hipGetErrorString(e));
        }
    }
    okpz::LatticeView v{s->buf[s->cur], (int32_t)s->Lx, (int32_t)s->Ly, s->W, s->ox};
    HIP_TRY(okpz::launch_width_rows(v, s->d_rows, s->stream));
    HIP_TRY(okpz::launch_psd(v, p, s->d_rows, s->psd_mem, s->stream));
    const double *spec =
        reinterpret_cast<const double *>(static_cast<const char *>(s->psd_mem) + p.off_spec);
    const size_t nx = (size_t)s->Lx / 2 + 1, ny = (size_t)s->Ly / 2 + 1;
    if (sx) HIP_TRY(hipMemcpyAsync(sx, spec, nx * 8, hipMemcpyDeviceToHost, s->stream));
    if (sy) HIP_TRY(hipMemcpyAsync(sy, spec + nx, ny * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return OKPZ_OK;
}

int okpz_psd_noalloc(okpz_sim *s, double *sx, double *sy)
{
    if (!s) return fail(OKPZ_EINVAL, "null handle");
    if (s->Lx > kStaticPsdMaxSide || s->Ly > kStaticPsdMaxSide)
        return fail(OKPZ_EINVAL,
                    "okpz_psd_noalloc: lattice %lldx%lld exceeds the static scratch's limit of "
                    "%lld sites per side",
                    (long long)s->Lx, (long long)s->Ly, (long long)kStaticPsdMaxSide);
    const okpz::PsdPlan p = okpz::psd_plan_capped(s->Lx, s->Ly, kStaticPsdBytes);
    if (p.bytes > kStaticPsdBytes)
        return fail(OKPZ_EINVAL, "okpz_psd_noalloc: %zu bytes of scratch needed, %zu available",
                    p.bytes, kStaticPsdBytes);
    hipError_t se;
    void *mem = static_scratch(s->device, &se);
    if (!mem) return hip_fail(se, "hipGetSymbolAddress(scratch)");
    okpz::LatticeView v{s->buf[s->cur], (int32_t)s->Lx, (int32_t)s->Ly, s->W, s->ox};
    HIP_TRY(okpz::launch_width_rows(v, s->d_rows, s->stream));
    HIP_TRY(okpz::launch_psd(v, p, s->d_rows, mem, s->stream));
    const double *spec = reinterpret_cast<const double *>(static_cast<const char *>(mem) + p.off_spec);
    const size_t nx = (size_t)s->Lx / 2 + 1, ny = (size_t)s->Ly / 2 + 1;
    if (sx) HIP_TRY(hipMemcpyAsync(sx, spec, nx * 8, hipMemcpyDeviceToHost, s->stream));
    if (sy) HIP_TRY(hipMemcpyAsync(sy, spec + nx, ny * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return OKPZ_OK;
}

int okpz_time(const okpz_sim *s, int64_t *t)
{
    if (!s || !t) return fail(OKPZ_EINVAL, "null argument");
    *t = s->t;
    return OKPZ_OK;
}

int okpz_h0(okpz_sim *s, int64_t *h0)
{
    if (!s || !h0) return fail(OKPZ_EINVAL, "null argument");
    HIP_TRY(hipMemcpyAsync(h0, s->d_h0, sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return OKPZ_OK;
}

void *okpz_stream(const okpz_sim *s) { return s ? reinterpret_cast<void *>(s->stream) : nullptr; }

int okpz_get_rows(okpz_sim *s, int64_t y0, int64_t nrows, uint8_t *host, size_t bytes)
{
    if (!s || !host) return fail(OKPZ_EINVAL, "null argument");
    if (nrows < 0 || nrows > s->Ly) return fail(OKPZ_EINVAL, "nrows out of range");
    if (bytes < (size_t)(nrows * s->Lx)) return fail(OKPZ_EINVAL, "host buffer too small");
    y0 = ((y0 % s->Ly) + s->Ly) % s->Ly;
    std::vector<uint32_t> p0, p1;
    int rc = download_rows(s, y0, nrows, p0, p1);
    if (rc != OKPZ_OK) return rc;
    unpack_rows(s, nrows, p0, p1, host);
    return OKPZ_OK;
}

int okpz_get_lattice(okpz_sim *s, uint8_t *host, size_t bytes)
{
    if (!s) return fail(OKPZ_EINVAL, "null handle");
    return okpz_get_rows(s, 0, s->Ly, host, bytes);
}

int okpz_set_lattice(okpz_sim *s, const uint8_t *host, size_t bytes, int64_t H0, int64_t t)
{
    if (!s || !host) return fail(OKPZ_EINVAL, "null argument");
    if (bytes < (size_t)(s->Lx * s->Ly)) return fail(OKPZ_EINVAL, "host buffer too small");
    if (t < 0 || t >= (int64_t(1) << 32)) return fail(OKPZ_EINVAL, "t out of range");
    if (!okpz::host::valid_h0(H0))
        return fail(OKPZ_EINVAL, "height of site (0,0) must be even (h = x + y mod 2)");
    std::string why;
    if (!okpz::host::valid_slope_field(host, s->Lx, s->Ly, why))
        return fail(OKPZ_EINVAL, "not a valid slope field: %s", why.c_str());
    int rc = upload_lattice(s, host);
    if (rc != OKPZ_OK) return rc;
    hipLaunchKernelGGL(set_h0_kernel, dim3(1), dim3(1), 0, s->stream, s->d_h0, H0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->t = t;
    return OKPZ_OK;
}

int okpz_save(okpz_sim *s, void *buf, size_t *bytes)
{
    if (!s || !bytes) return fail(OKPZ_EINVAL, "null argument");
    const size_t pb = plane_bytes(s->Lx, s->Ly);
    const size_t need = sizeof(CkptHeader) + pb;
    if (!buf) {
        *bytes = need;
        return OKPZ_OK;
    }
    if (*bytes < need) return fail(OKPZ_EINVAL, "checkpoint buffer too small (%zu < %zu)", *bytes, need);
    int64_t H0;
    int rc = okpz_h0(s, &H0);
    if (rc != OKPZ_OK) return rc;
    CkptHeader h{};
    std::memcpy(h.magic, "OKPZCKP1", 8);
    h.version = 1;
    h.cell_borders = (uint32_t)s->cell_borders;
    h.Lx = s->Lx;
    h.Ly = s->Ly;
    h.p = s->p;
    h.q = s->q;
    h.seed = s->seed;
    h.t = s->t;
    h.H0 = H0;
    h.ox = s->ox;
    h.copies = s->copies;
    std::memcpy(buf, &h, sizeof h);
    HIP_TRY(hipMemcpy(static_cast<char *>(buf) + sizeof h, s->buf[s->cur], pb, hipMemcpyDeviceToHost));
    *bytes = need;
    return OKPZ_OK;
}

int okpz_load(okpz_sim **out, const void *buf, size_t bytes)
{
    if (!out || !buf) return fail(OKPZ_EINVAL, "null argument");
    *out = nullptr;
    CkptHeader h;
    const uint32_t *planes = nullptr;
    std::string why;
    if (!okpz::host::parse_checkpoint(buf, bytes, &h, &planes, why))
        return fail(OKPZ_EINVAL, "%s", why.c_str());
    const size_t pb = plane_bytes(h.Lx, h.Ly);
    okpz_sim *s = nullptr;
    int rc = make_sim(&s, h.Lx, h.Ly, h.p, h.q, h.seed, nullptr, 0, nullptr, h.copies == 1 ? 1 : 2);
    if (rc != OKPZ_OK) return rc;
    hipError_t e = hipMemcpy(s->buf[0], planes, pb, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release(s);
        return hip_fail(e, "hipMemcpy(checkpoint)");
    }
    hipLaunchKernelGGL(set_h0_kernel, dim3(1), dim3(1), 0, s->stream, s->d_h0, h.H0);
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        release(s);
        return hip_fail(e, "restore");
    }
    s->cur = 0;
    s->ox = h.ox;
    s->t = h.t;
    s->cell_borders = (int32_t)h.cell_borders;
    *out = s;
    return OKPZ_OK;
}

int okpz_set_cell_borders(okpz_sim *s, int32_t kind)
{
    if (!s) return fail(OKPZ_EINVAL, "null handle");
    if (kind != OKPZ_CELLS_DEAD && kind != OKPZ_CELLS_DELAYED)
        return fail(OKPZ_EINVAL, "cell border kind %d is neither dead (0) nor delayed (1)", kind);
    s->cell_borders = kind;
    return OKPZ_OK;
}

int okpz_get_cell_borders(const okpz_sim *s, int32_t *kind)
{
    if (!s || !kind) return fail(OKPZ_EINVAL, "null argument");
    *kind = s->cell_borders;
    return OKPZ_OK;
}

int okpz_set_threads(okpz_sim *s, int threads)
{
    if (!s) return fail(OKPZ_EINVAL, "null handle");
    if (!okpz::sweep_threads_ok(threads))
        return fail(OKPZ_EINVAL, "threads per workgroup must be 256, 512 or 1024");
    s->threads = threads;
    return OKPZ_OK;
}

int okpz_sync(okpz_sim *s)
{
    if (!s) return fail(OKPZ_EINVAL, "null handle");
    HIP_TRY(hipStreamSynchronize(s->stream));
    return OKPZ_OK;
}

int okpz_free(okpz_sim *s)
{
    if (!s) return OKPZ_OK;
    release(s);
    return OKPZ_OK;
}

int okpz_sampling_times(int64_t t_max, double m, int64_t *times, int64_t cap, int64_t *n)
{
    if (!n) return fail(OKPZ_EINVAL, "null argument");
    if (!(m > 0.0) || m > 10.0) return fail(OKPZ_EINVAL, "sampling exponent m must be in (0, 10]");
    if (t_max < 0 || t_max >= (int64_t(1) << 32)) return fail(OKPZ_EINVAL, "t_max out of range");
    const std::vector<int64_t> v = okpz::host::sample_times(t_max, m);
    *n = (int64_t)v.size();
    if (times) {
        if (cap < *n) return fail(OKPZ_EINVAL, "%lld times need room, %lld given", (long long)*n, (long long)cap);
        std::copy(v.begin(), v.end(), times);
    }
    return OKPZ_OK;
}

const char *okpz_last_error(void) { return g_err.c_str(); }

}  // extern "C"
