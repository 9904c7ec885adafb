// Batched ensembles on gfx950: many independent realizations of uneven size,
// each with its own p, q, seed and length, run to completion in ONE
// persistent launch (ensembles of independent runs, Sec. III and IV).
//
// Work item = (job, group of blocks) of the job's current sweep.  Resident
// workgroups take items from a bounded multi-producer multi-consumer ring in
// device memory; the workgroup that completes the last group of a job's sweep
// advances the job (time, stored offset, lattice copy), measures the exact
// width when a sampling time is reached, and enqueues the job's next sweep.
// No workgroup ever waits for a particular other workgroup, so the launch
// needs no co-residency; a workgroup that finds the ring empty sleeps
// briefly and retries, and a global progress counter acts as watchdog: if no
// group completes anywhere for a long time every workgroup exits with an
// error flag instead of spinning forever.
//
// Memory ordering: lattice words written by one workgroup are read by the
// next sweep's workgroups on any XCD; each group completion releases at agent
// scope (writes back the XCD's L2) and every dequeue acquires at agent scope.
//
// A job's trajectory is identical to the same job run alone through
// okpz_sweep: the random decisions are keyed by (seed, sweep, block, step,
// cell) and the groups only decide which workgroup does the work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "okpz.h"
#include "sweep_core.h"
#include "width_core.h"

namespace okpz {
namespace batch {

struct JobDesc {
    uint32_t *buf[2];
    int64_t *h0;
    int64_t *rows;      // width scratch, 3 * Ly
    int64_t *samples;   // nsamp x 6: t, S1' lo, S1' hi, S2' lo, S2' hi, H0
    const int32_t *sample_t;
    int32_t nsamp;
    int32_t Lx, Ly, W, Bx, By, nbx, nby, G, ngroups, mode;
    int32_t t_max;
    uint32_t k0, k1;
    uint64_t Tp, Tq;
};

struct JobState {
    int32_t s;            // sweep in progress (= MCS completed)
    int32_t ox;           // stored offset of the source copy
    int32_t cur;          // source copy
    int32_t next_sample;  // index of the next sampling time
    uint32_t done;        // groups of sweep s completed
    int32_t pad[3];
};

struct Control {
    uint64_t head, tail;  // ring positions
    uint64_t progress;    // groups completed by the whole launch
    int32_t finished;     // jobs that reached t_max
    int32_t error;        // 1: watchdog, 2: ring full
};

__device__ __forceinline__ uint64_t ld_acq(uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rlx(uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas(uint64_t *p, uint64_t &expect, uint64_t want)
{
    return __hip_atomic_compare_exchange_strong(p, &expect, want, __ATOMIC_ACQ_REL,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded MPMC ring (sequence-numbered cells).  Returns false if full.
__device__ bool enqueue(Control *c, uint64_t *seq, uint64_t *val, uint64_t mask, uint64_t item)
{
    uint64_t pos = ld_rlx(&c->tail);
    for (int tries = 0; tries < (1 << 20); ++tries) {
        const uint64_t sq = ld_acq(&seq[pos & mask]);
        const int64_t dif = (int64_t)(sq - pos);
        if (dif == 0) {
            if (cas(&c->tail, pos, pos + 1)) {
                __hip_atomic_store(&val[pos & mask], item, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                st_rel(&seq[pos & mask], pos + 1);
                return true;
            }
        } else if (dif < 0) {
            return false;
        } else {
            pos = ld_rlx(&c->tail);
        }
    }
    return false;
}

// Returns true and the item, or false if the ring is empty.
__device__ bool dequeue(Control *c, uint64_t *seq, uint64_t *val, uint64_t mask, uint64_t *item)
{
    uint64_t pos = ld_rlx(&c->head);
    for (int tries = 0; tries < (1 << 20); ++tries) {
        const uint64_t sq = ld_acq(&seq[pos & mask]);
        const int64_t dif = (int64_t)(sq - (pos + 1));
        if (dif == 0) {
            if (cas(&c->head, pos, pos + 1)) {
                *item = __hip_atomic_load(&val[pos & mask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                st_rel(&seq[pos & mask], pos + mask + 1);
                return true;
            }
        } else if (dif < 0) {
            return false;
        } else {
            pos = ld_rlx(&c->head);
        }
    }
    return false;
}

__device__ inline SweepLaunch make_launch(const JobDesc &jd, const JobState &js)
{
    SweepLaunch a{};
    a.src = js.cur ? jd.buf[1] : jd.buf[0];  // (selects, not a dynamic index)
    a.dst = js.cur ? jd.buf[0] : jd.buf[1];
    a.h0 = jd.h0;
    a.Lx = jd.Lx;
    a.Ly = jd.Ly;
    a.W = jd.W;
    a.Bx = jd.Bx;
    a.By = jd.By;
    a.nbx = jd.nbx;
    a.nby = jd.nby;
    a.ox_src = js.ox;
    a.s = (uint32_t)js.s;
    a.k0 = jd.k0;
    a.k1 = jd.k1;
    a.Tp = jd.Tp;
    a.Tq = jd.Tq;
    const Ctr4 r = philox10(Ctr4{a.s, 0, 0, kTagShift}, a.k0, a.k1);
    a.sx = (int32_t)below(r.x, (uint32_t)jd.Bx);
    a.sy = (int32_t)below(r.y, (uint32_t)jd.By);
    const int x00 = (jd.Lx - a.sx) % jd.Lx, y00 = (jd.Ly - a.sy) % jd.Ly;
    a.blk00 = (y00 / jd.By) * jd.nbx + x00 / jd.Bx;
    a.u00 = x00 % jd.Bx;
    a.v00 = y00 % jd.By;
    return a;
}

template <int kThreads, int kMode>
__device__ __forceinline__ void run_group(const SweepLaunch &a, int b0, int G, uint8_t *smem)
{
    const int tiles = ((G * (a.By + 1) * a.Bx) + 15) & ~15;
    uint32_t *opk = reinterpret_cast<uint32_t *>(smem + tiles);
    if (a.Bx == core::kMaxB && a.By == core::kMaxB)
        core::sweep_group<kThreads, kMode, core::kMaxB>(a, b0, 1, smem, opk);
    else
        core::sweep_group<kThreads, kMode, 0>(a, b0, G, smem, opk);
}

// Publish job r's next sweep (or count it finished).  Thread 0 only.
__device__ void advance(const JobDesc &jd, JobState *js, Control *ctl, uint64_t *qseq,
                        uint64_t *qval, uint64_t qmask, int r)
{
    if (js->s >= jd.t_max) {
        __hip_atomic_fetch_add(&ctl->finished, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    __atomic_thread_fence(__ATOMIC_RELEASE);
    for (int g = 0; g < jd.ngroups; ++g) {
        if (!enqueue(ctl, qseq, qval, qmask, ((uint64_t)r << 32) | (uint32_t)g)) {
            __hip_atomic_store(&ctl->error, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
    }
}

template <int kThreads>
__global__ __launch_bounds__(kThreads) void batch_kernel(const JobDesc *jobs, JobState *state,
                                                         Control *ctl, uint64_t *qseq, uint64_t *qval,
                                                         uint64_t qmask, int32_t njobs,
                                                         uint64_t idle_limit)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint64_t s_item;
    __shared__ int s_cmd;    // 0: work, 1: exit, 2: retry
    __shared__ int s_width;  // 1: the job just reached a sampling time
    __shared__ int64_t s_out[4];
    const int tid = threadIdx.x;
    uint64_t idle = 0, seen = 0;

    while (true) {
        if (tid == 0) {
            uint64_t item = 0;
            int cmd = 2;
            if (dequeue(ctl, qseq, qval, qmask, &item)) {
                cmd = 0;
                idle = 0;
            } else if (__hip_atomic_load(&ctl->finished, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= njobs ||
                       __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                cmd = 1;
            } else {
                const uint64_t p = ld_rlx(&ctl->progress);
                if (p != seen) {
                    seen = p;
                    idle = 0;
                } else if (++idle > idle_limit) {
                    __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    cmd = 1;
                }
                __builtin_amdgcn_s_sleep(8);
            }
            s_item = item;
            s_cmd = cmd;
        }
        __syncthreads();
        const int cmd = s_cmd;
        const uint64_t item = s_item;
        __syncthreads();
        if (cmd == 1) break;
        if (cmd == 2) continue;

        __atomic_thread_fence(__ATOMIC_ACQUIRE);  // every thread: see the job's state and lattice
        const int r = (int)(item >> 32), gi = (int)(item & 0xffffffffu);
        const JobDesc jd = jobs[r];
        const JobState js = state[r];
        const SweepLaunch a = make_launch(jd, js);
        const int b0 = gi * jd.G;
        const int Gc = min(jd.G, jd.nbx * jd.nby - b0);
        if (jd.mode == core::kGrowth)
            run_group<kThreads, core::kGrowth>(a, b0, Gc, smem);
        else if (jd.mode == core::kFixed)
            run_group<kThreads, core::kFixed>(a, b0, Gc, smem);
        else
            run_group<kThreads, core::kDraw>(a, b0, Gc, smem);
        __syncthreads();

        if (tid == 0) {
            s_width = 0;
            __atomic_thread_fence(__ATOMIC_RELEASE);
            __hip_atomic_fetch_add(&ctl->progress, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t d = __hip_atomic_fetch_add(&state[r].done, 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_AGENT) + 1u;
            if (d == (uint32_t)jd.ngroups) {  // last group of sweep s: advance the job
                JobState ns = js;
                ns.s = js.s + 1;
                ns.ox = a.sx;
                ns.cur = js.cur ^ 1;
                ns.done = 0;
                const bool sample = ns.next_sample < jd.nsamp && jd.sample_t[ns.next_sample] == ns.s;
                state[r] = ns;
                if (sample)
                    s_width = 1;
                else
                    advance(jd, &state[r], ctl, qseq, qval, qmask, r);
            }
        }
        __syncthreads();
        if (s_width) {
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
            const JobState ns = state[r];
            const LatticeView v{ns.cur ? jd.buf[1] : jd.buf[0], jd.Lx, jd.Ly, jd.W, ns.ox};
            const int lane = tid & 63, wave = tid >> 6, nwave = kThreads / 64;
            for (int y = wave; y < jd.Ly; y += nwave) core::width_row(v, y, lane, jd.rows);
            __atomic_thread_fence(__ATOMIC_RELEASE);
            __syncthreads();
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
            int32_t *scan = reinterpret_cast<int32_t *>(smem);
            int64_t *r1 = reinterpret_cast<int64_t *>(smem + 4 * 1024);
            int64_t *r2 = reinterpret_cast<int64_t *>(smem + 12 * 1024);
            core::width_combine(jd.rows, jd.Lx, jd.Ly, s_out, scan, r1, r2);
            if (tid == 0) {
                int64_t *o = jd.samples + 6 * (size_t)ns.next_sample;
                o[0] = ns.s;
                o[1] = s_out[0];
                o[2] = s_out[1];
                o[3] = s_out[2];
                o[4] = s_out[3];
                o[5] = __hip_atomic_load(jd.h0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                state[r].next_sample = ns.next_sample + 1;
                advance(jd, &state[r], ctl, qseq, qval, qmask, r);
            }
            __syncthreads();
        }
    }
}

__global__ void init_jobs_kernel(const JobDesc *jobs, int32_t njobs)
{
    // flat zig-zag state h = (x+y) mod 2 in copy 0 of every job, H0 = 0
    const int r = blockIdx.y;
    if (r >= njobs) return;
    const JobDesc jd = jobs[r];
    const size_t n = 2 * (size_t)jd.Ly * jd.W;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t y = (e / jd.W) % jd.Ly;
        jd.buf[0][e] = (y & 1) ? 0xAAAAAAAAu : 0x55555555u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *jd.h0 = 0;
}

}  // namespace batch
}  // namespace okpz

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
using okpz::batch::Control;
using okpz::batch::JobDesc;
using okpz::batch::JobState;

struct okpz_batch {
    std::vector<okpz_job> jobs;
    std::vector<std::vector<int32_t>> times;
    std::vector<JobDesc> desc;
    double m;
    void *mem = nullptr;
    JobDesc *d_desc = nullptr;
    JobState *d_state = nullptr;
    Control *d_ctl = nullptr;
    uint64_t *d_qseq = nullptr, *d_qval = nullptr;
    uint64_t qcap = 0;
    int threads = 1024;
    int workgroups = 0;  // 0: two per compute unit
    int cus = 0;
    hipStream_t stream = nullptr;
    bool ran = false;
    float last_ms = 0.f;
};

namespace {

thread_local std::string b_err;

int bfail(int code, const char *fmt, ...)
{
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    b_err = msg;
    return code;
}

#define BHIP(expr)                                                                 \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) return bfail(OKPZ_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool side_ok(int64_t L) { return L >= 32 && L <= 8192 && L % 32 == 0; }

std::vector<int32_t> sample_times(int64_t t_max, double m)
{
    std::vector<int32_t> out;
    if (t_max <= 0) return out;
    double t = 0.0;
    while (true) {
        t = (t + 10.0) * std::exp(m);
        if (t > (double)t_max) break;
        const int32_t c = (int32_t)std::ceil(t);
        if (out.empty() || out.back() != c) out.push_back(c);
    }
    if (out.empty() || out.back() != t_max) out.push_back((int32_t)t_max);
    return out;
}

size_t al(size_t n) { return (n + 255) / 256 * 256; }

// (Re)start every job from the flat state with the given sweep limit.
int reset(okpz_batch *b, const std::vector<int32_t> &tmax)
{
    const int n = (int)b->jobs.size();
    std::vector<JobState> st(n);
    std::memset(st.data(), 0, st.size() * sizeof(JobState));
    std::vector<JobDesc> desc = b->desc;
    uint64_t n0 = 0;
    std::vector<uint64_t> qseq(b->qcap), qval(b->qcap, 0);
    for (int r = 0; r < n; ++r) {
        desc[r].t_max = tmax[r];
        // sampling times beyond the limit are not reached
        int ns = 0;
        while (ns < (int)b->times[r].size() && b->times[r][ns] <= tmax[r]) ++ns;
        desc[r].nsamp = ns;
    }
    int finished = 0;
    for (int r = 0; r < n; ++r) {
        if (desc[r].t_max == 0) {
            ++finished;
            continue;
        }
        for (int g = 0; g < desc[r].ngroups; ++g) {
            qval[n0] = ((uint64_t)r << 32) | (uint32_t)g;
            ++n0;
        }
    }
    for (uint64_t i = 0; i < b->qcap; ++i) qseq[i] = (i < n0) ? i + 1 : i;
    Control ctl{};
    ctl.head = 0;
    ctl.tail = n0;
    ctl.finished = finished;
    BHIP(hipMemcpyAsync(b->d_desc, desc.data(), n * sizeof(JobDesc), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_state, st.data(), n * sizeof(JobState), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_qseq, qseq.data(), b->qcap * 8, hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_qval, qval.data(), b->qcap * 8, hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, b->stream));
    int maxwords = 0;
    for (auto &d : desc) maxwords = std::max(maxwords, 2 * d.Ly * d.W);
    const int bx = std::min(4096, (maxwords + 255) / 256);
    hipLaunchKernelGGL(okpz::batch::init_jobs_kernel, dim3(bx, n), dim3(256), 0, b->stream, b->d_desc, n);
    BHIP(hipGetLastError());
    BHIP(hipStreamSynchronize(b->stream));
    return OKPZ_OK;
}

template <int kThreads>
hipError_t launch_batch(okpz_batch *b, int wgs)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)okpz::batch::batch_kernel<kThreads>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           okpz::core::kGroupLds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    // about 2 s without any group completing anywhere (one probe: a dequeue
    // attempt plus a sleep of 8 x 64 cycles)
    const uint64_t idle_limit = 1ull << 20;
    hipLaunchKernelGGL((okpz::batch::batch_kernel<kThreads>), dim3(wgs), dim3(kThreads),
                       okpz::core::kGroupLds, b->stream, b->d_desc, b->d_state, b->d_ctl, b->d_qseq,
                       b->d_qval, b->qcap - 1, (int32_t)b->jobs.size(), idle_limit);
    return hipGetLastError();
}

int run(okpz_batch *b, int threads, int wgs, float *ms)
{
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    BHIP(hipEventRecord(e0, b->stream));
    hipError_t e;
    switch (threads) {
    case 256: e = launch_batch<256>(b, wgs); break;
    case 512: e = launch_batch<512>(b, wgs); break;
    default: e = launch_batch<1024>(b, wgs); break;
    }
    if (e != hipSuccess) return bfail(OKPZ_EDEVICE, "batch launch: %s", hipGetErrorString(e));
    BHIP(hipEventRecord(e1, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    float t = 0.f;
    BHIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms) *ms = t;
    Control ctl;
    BHIP(hipMemcpy(&ctl, b->d_ctl, sizeof ctl, hipMemcpyDeviceToHost));
    if (ctl.error == 1) return bfail(OKPZ_EDEVICE, "batch watchdog: no progress (finished %d of %zu)",
                                     ctl.finished, b->jobs.size());
    if (ctl.error == 2) return bfail(OKPZ_EDEVICE, "batch work ring overflow");
    if (ctl.finished != (int)b->jobs.size())
        return bfail(OKPZ_EDEVICE, "batch ended with %d of %zu jobs finished", ctl.finished,
                     b->jobs.size());
    return OKPZ_OK;
}

}  // namespace

extern "C" {

int okpz_batch_create(okpz_batch **out, const okpz_job *jobs, int32_t n_jobs, double m)
{
    if (!out) return bfail(OKPZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (!jobs || n_jobs <= 0 || n_jobs > 65535) return bfail(OKPZ_EINVAL, "need 1 .. 65535 jobs");
    if (!(m > 0.0) || m > 10.0) return bfail(OKPZ_EINVAL, "sampling exponent m must be in (0, 10]");
    for (int r = 0; r < n_jobs; ++r) {
        const okpz_job &j = jobs[r];
        if (!side_ok(j.Lx) || !side_ok(j.Ly))
            return bfail(OKPZ_EINVAL, "job %d: sides must be multiples of 32 in [32, 8192]", r);
        if (!(j.p >= 0.0 && j.p <= 1.0) || !(j.q >= 0.0 && j.q <= 1.0))
            return bfail(OKPZ_EINVAL, "job %d: p and q must lie in [0,1]", r);
        if (j.t_max < 0 || j.t_max >= (int64_t(1) << 31))
            return bfail(OKPZ_EINVAL, "job %d: t_max out of range", r);
    }
    okpz_batch *b = new okpz_batch();
    b->jobs.assign(jobs, jobs + n_jobs);
    b->m = m;
    b->times.resize(n_jobs);
    b->desc.resize(n_jobs);
    // layout: descriptors, states, control, ring, then per-job lattices etc.
    size_t total = al(n_jobs * sizeof(JobDesc)) + al(n_jobs * sizeof(JobState)) + al(sizeof(Control));
    uint64_t groups = 0;
    std::vector<size_t> offs(n_jobs);
    for (int r = 0; r < n_jobs; ++r) {
        const okpz_job &j = jobs[r];
        okpz::Geometry g;
        okpz::geometry_of(j.Lx, j.Ly, &g);
        const int nbx = (int)(j.Lx / g.Bx), nby = (int)(j.Ly / g.By);
        const int G = okpz::core::group_size(g.Bx, g.By, nbx * nby);
        JobDesc &d = b->desc[r];
        std::memset(&d, 0, sizeof d);
        d.Lx = (int32_t)j.Lx;
        d.Ly = (int32_t)j.Ly;
        d.W = (int32_t)(j.Lx / 32);
        d.Bx = g.Bx;
        d.By = g.By;
        d.nbx = nbx;
        d.nby = nby;
        d.G = G;
        d.ngroups = (nbx * nby + G - 1) / G;
        d.k0 = (uint32_t)(j.seed & 0xffffffffu);
        d.k1 = (uint32_t)(j.seed >> 32);
        d.Tp = okpz::threshold_of(j.p);
        d.Tq = okpz::threshold_of(j.q);
        const uint64_t one = uint64_t(1) << 32;
        const bool trivial = (d.Tp == 0 || d.Tp == one) && (d.Tq == 0 || d.Tq == one);
        d.mode = !trivial ? okpz::core::kDraw
                          : (d.Tp == one && d.Tq == 0 ? okpz::core::kGrowth : okpz::core::kFixed);
        d.t_max = (int32_t)j.t_max;
        b->times[r] = sample_times(j.t_max, m);
        d.nsamp = (int32_t)b->times[r].size();
        groups += d.ngroups;
        offs[r] = total;
        const size_t lat = al(2 * (size_t)j.Ly * (size_t)(j.Lx / 32) * 4);
        total += 2 * lat + al(8) + al(3 * (size_t)j.Ly * 8) + al(6 * 8 * (size_t)std::max(1, d.nsamp)) +
                 al(4 * (size_t)std::max(1, d.nsamp));
    }
    b->qcap = 1;
    while (b->qcap < groups + 1) b->qcap <<= 1;
    const size_t qoff = total;
    total += 2 * al(b->qcap * 8);
    hipError_t e = hipMalloc(&b->mem, total);
    if (e != hipSuccess) {
        delete b;
        return bfail(OKPZ_ENOMEM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
    }
    char *base = static_cast<char *>(b->mem);
    b->d_desc = reinterpret_cast<JobDesc *>(base);
    b->d_state = reinterpret_cast<JobState *>(base + al(n_jobs * sizeof(JobDesc)));
    b->d_ctl = reinterpret_cast<Control *>(base + al(n_jobs * sizeof(JobDesc)) +
                                           al(n_jobs * sizeof(JobState)));
    b->d_qseq = reinterpret_cast<uint64_t *>(base + qoff);
    b->d_qval = reinterpret_cast<uint64_t *>(base + qoff + al(b->qcap * 8));
    for (int r = 0; r < n_jobs; ++r) {
        const okpz_job &j = jobs[r];
        JobDesc &d = b->desc[r];
        char *p = base + offs[r];
        const size_t lat = al(2 * (size_t)j.Ly * (size_t)(j.Lx / 32) * 4);
        d.buf[0] = reinterpret_cast<uint32_t *>(p);
        d.buf[1] = reinterpret_cast<uint32_t *>(p + lat);
        d.h0 = reinterpret_cast<int64_t *>(p + 2 * lat);
        d.rows = reinterpret_cast<int64_t *>(p + 2 * lat + al(8));
        d.samples = reinterpret_cast<int64_t *>(p + 2 * lat + al(8) + al(3 * (size_t)j.Ly * 8));
        int32_t *tt = reinterpret_cast<int32_t *>(p + 2 * lat + al(8) + al(3 * (size_t)j.Ly * 8) +
                                                   al(6 * 8 * (size_t)std::max(1, d.nsamp)));
        d.sample_t = tt;
        if (d.nsamp) {
            e = hipMemcpy(tt, b->times[r].data(), d.nsamp * 4, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(b->mem);
                delete b;
                return bfail(OKPZ_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
            }
        }
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (b->cus <= 0) b->cus = 256;
    e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(b->mem);
        delete b;
        return bfail(OKPZ_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    *out = b;
    return OKPZ_OK;
}

int okpz_batch_set_mapping(okpz_batch *b, int32_t threads, int32_t workgroups)
{
    if (!b) return bfail(OKPZ_EINVAL, "null batch");
    if (threads != 256 && threads != 512 && threads != 1024)
        return bfail(OKPZ_EINVAL, "threads per workgroup must be 256, 512 or 1024");
    if (workgroups < 0 || workgroups > (1 << 16)) return bfail(OKPZ_EINVAL, "workgroups out of range");
    b->threads = threads;
    b->workgroups = workgroups;
    return OKPZ_OK;
}

int okpz_batch_get_mapping(okpz_batch *b, int32_t *threads, int32_t *workgroups)
{
    if (!b) return bfail(OKPZ_EINVAL, "null batch");
    if (threads) *threads = b->threads;
    if (workgroups) *workgroups = b->workgroups ? b->workgroups : 2 * b->cus;
    return OKPZ_OK;
}

int okpz_batch_run(okpz_batch *b)
{
    if (!b) return bfail(OKPZ_EINVAL, "null batch");
    std::vector<int32_t> tmax(b->jobs.size());
    for (size_t r = 0; r < b->jobs.size(); ++r) tmax[r] = (int32_t)b->jobs[r].t_max;
    int rc = reset(b, tmax);
    if (rc != OKPZ_OK) return rc;
    const int wgs = b->workgroups ? b->workgroups : 2 * b->cus;
    rc = run(b, b->threads, wgs, &b->last_ms);
    if (rc == OKPZ_OK) b->ran = true;
    return rc;
}

int okpz_batch_last_ms(okpz_batch *b, float *ms)
{
    if (!b || !ms) return bfail(OKPZ_EINVAL, "null argument");
    *ms = b->last_ms;
    return OKPZ_OK;
}

int okpz_batch_autotune(okpz_batch *b, int64_t trial_mcs, int32_t *threads, int32_t *workgroups)
{
    if (!b) return bfail(OKPZ_EINVAL, "null batch");
    if (trial_mcs <= 0) return bfail(OKPZ_EINVAL, "trial_mcs must be positive");
    std::vector<int32_t> tmax(b->jobs.size());
    for (size_t r = 0; r < b->jobs.size(); ++r)
        tmax[r] = (int32_t)std::min<int64_t>(b->jobs[r].t_max, trial_mcs);
    const int cand_t[3] = {1024, 512, 256};
    const int cand_w[2] = {2 * b->cus, b->cus};
    float best = 1e30f;
    int bt = b->threads, bw = b->workgroups;
    for (int ti = 0; ti < 3; ++ti)
        for (int wi = 0; wi < 2; ++wi) {
            int rc = reset(b, tmax);
            if (rc != OKPZ_OK) return rc;
            float ms = 0.f;
            rc = run(b, cand_t[ti], cand_w[wi], &ms);
            if (rc != OKPZ_OK) return rc;
            if (ms < best) {
                best = ms;
                bt = cand_t[ti];
                bw = cand_w[wi];
            }
        }
    b->threads = bt;
    b->workgroups = bw;
    b->ran = false;
    if (threads) *threads = bt;
    if (workgroups) *workgroups = bw;
    return OKPZ_OK;
}

int okpz_batch_samples(okpz_batch *b, int32_t job, int64_t *t, int64_t *sum_h, int64_t *sum_h2,
                       int32_t cap, int32_t *count)
{
    if (!b || !count) return bfail(OKPZ_EINVAL, "null argument");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return bfail(OKPZ_EINVAL, "job out of range");
    if (!b->ran) return bfail(OKPZ_EINVAL, "batch has not been run");
    const JobDesc &d = b->desc[job];
    const int n = d.nsamp;
    *count = n;
    if (!t && !sum_h && !sum_h2) return OKPZ_OK;
    if (cap < n) return bfail(OKPZ_EINVAL, "capacity %d < %d samples", cap, n);
    std::vector<int64_t> raw(6 * (size_t)std::max(1, n));
    BHIP(hipMemcpy(raw.data(), d.samples, 6 * 8 * (size_t)n, hipMemcpyDeviceToHost));
    const __int128 N = (__int128)d.Lx * d.Ly;
    const __int128 lim = (__int128)1 << 63;
    for (int i = 0; i < n; ++i) {
        const int64_t *o = &raw[6 * (size_t)i];
        const __int128 s1r = (__int128)(((unsigned __int128)(uint64_t)o[2] << 64) | (uint64_t)o[1]);
        const __int128 s2r = (__int128)(((unsigned __int128)(uint64_t)o[4] << 64) | (uint64_t)o[3]);
        const __int128 H0 = o[5];
        const __int128 S1 = s1r + N * H0;
        const __int128 S2 = s2r + 2 * H0 * s1r + N * H0 * H0;
        if (S1 >= lim || S1 < -lim || S2 >= lim || S2 < 0)
            return bfail(OKPZ_EOVERFLOW, "job %d sample %d exceeds int64", job, i);
        if (t) t[i] = o[0];
        if (sum_h) sum_h[i] = (int64_t)S1;
        if (sum_h2) sum_h2[i] = (int64_t)S2;
    }
    return OKPZ_OK;
}

int okpz_batch_h0(okpz_batch *b, int32_t job, int64_t *h0)
{
    if (!b || !h0) return bfail(OKPZ_EINVAL, "null argument");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return bfail(OKPZ_EINVAL, "job out of range");
    BHIP(hipMemcpy(h0, b->desc[job].h0, 8, hipMemcpyDeviceToHost));
    return OKPZ_OK;
}

int okpz_batch_get_lattice(okpz_batch *b, int32_t job, uint8_t *host, size_t bytes)
{
    if (!b || !host) return bfail(OKPZ_EINVAL, "null argument");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return bfail(OKPZ_EINVAL, "job out of range");
    const JobDesc &d = b->desc[job];
    if (bytes < (size_t)d.Lx * d.Ly) return bfail(OKPZ_EINVAL, "host buffer too small");
    JobState st;
    BHIP(hipMemcpy(&st, b->d_state + job, sizeof st, hipMemcpyDeviceToHost));
    std::vector<uint32_t> pl(2 * (size_t)d.Ly * d.W);
    BHIP(hipMemcpy(pl.data(), d.buf[st.cur], pl.size() * 4, hipMemcpyDeviceToHost));
    for (int64_t y = 0; y < d.Ly; ++y)
        for (int64_t x = 0; x < d.Lx; ++x) {
            const int64_t c = ((x - st.ox) % d.Lx + d.Lx) % d.Lx;
            const uint32_t bx = (pl[(size_t)y * d.W + (c >> 5)] >> (c & 31)) & 1u;
            const uint32_t by = (pl[((size_t)d.Ly + y) * d.W + (c >> 5)] >> (c & 31)) & 1u;
            host[y * d.Lx + x] = (uint8_t)(bx | (by << 1));
        }
    return OKPZ_OK;
}

int okpz_batch_free(okpz_batch *b)
{
    if (!b) return OKPZ_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->mem) (void)hipFree(b->mem);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return OKPZ_OK;
}

const char *okpz_batch_last_error(void) { return b_err.c_str(); }

}  // extern "C"
