// Batched ensembles on gfx950: many independent realizations of uneven size,
// each with its own p, q, seed and length, run to completion in ONE
// persistent launch (ensembles of independent runs, Sec. III and IV).
//
// Work item = (job, chunk of groups of blocks) of the job's current sweep
// (one group per item for lattices up to 2048 x 2048; larger lattices hand
// out at most 128 items per sweep).  Each job has a claim word (sweep << 32 |
// next item); a resident workgroup's first wavefront scans the claim words,
// 64 jobs per load, and claims an item of a job with one fetch-and-add on
// that job's word, so contention is spread over the jobs.  The workgroup that
// completes the last item of a job's sweep advances the job (time, stored offset, lattice copy), measures the
// exact width when a sampling time is reached, and reopens the job's claim
// word for the next sweep.  No workgroup ever waits for a particular other
// workgroup, so the launch needs no co-residency; a workgroup that finds no
// open group sleeps briefly and rescans, and a global progress counter acts
// as watchdog: if no group completes anywhere for a long time every
// workgroup exits with an error flag instead of spinning forever.
//
// Memory ordering: lattice words written by one workgroup are read by the
// next sweep's workgroups on any XCD.  Scans are relaxed loads; a successful
// claim is followed by one agent-scope acquire, a completed group by one
// acquire-release count, and a reopened job by one release.
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

#include "host_logic.h"
#include "okpz.h"
#include "sweep_core.h"
#include "width.h"
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
    int32_t chunk;   // groups per work item
    int32_t nitems;  // work items per sweep
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
    uint64_t progress;  // sweeps completed by the whole launch
    int32_t finished;   // jobs that reached their stop target
    int32_t error;      // 1: watchdog
};

// claim[r] = (sweep << 32) | next item to hand out; job r has an open item
// while the low word is below nitems[r] (its items per sweep).  A finished or empty job holds
// kClosed in the low word.  A scan can see a word open that is exhausted or
// closed by the time the wave's fetch-and-add lands; such late increments
// are at most two (one claim) per workgroup per word value, so the low word
// never carries into the sweep number (kClosed + 2 workgroups < 2^32).
constexpr uint32_t kClosed = 0x80000000u;

// Polled words (claim words, counters) are read and published at system
// scope, which bypasses the per-XCD caches: a poller never spins on a stale
// line.
__device__ __forceinline__ uint64_t ld_rlx(uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
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
    uint32_t *opk = reinterpret_cast<uint32_t *>(smem + core::tile_bytes(a.Bx, a.By, G));
    if (a.Bx == core::kMaxB && a.By == core::kMaxB)
        core::sweep_group<kThreads, kMode, core::kMaxB, true>(a, b0, 1, smem, opk);
    else if (a.Bx * a.By >= 128 * 128)  // a wave's cells share a block
        core::sweep_group<kThreads, kMode, 0, true, false>(a, b0, G, smem, opk);
    else
        core::sweep_group<kThreads, kMode, 0, true, true>(a, b0, G, smem, opk);
}

// Publish job r's next sweep (or count it finished).  Thread 0 only, after
// the job's state for the new sweep has been written.
__device__ void publish(const JobDesc &jd, const JobState &ns, Control *ctl, uint64_t *claim, int r)
{
    // one completed sweep: the watchdog's sign of life
    __hip_atomic_fetch_add(&ctl->progress, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ns.s >= jd.t_max) {
        __hip_atomic_store(&claim[r], ((uint64_t)ns.s << 32) | kClosed, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_fetch_add(&ctl->finished, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // state and lattice before the claim word
    __hip_atomic_store(&claim[r], (uint64_t)ns.s << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Claim policy of a launch (flags):
//   kClaimPairs: a workgroup takes two items of a job whose sweep has at
//     least eight, so such a job still spreads over four or more workgroups
//     while its claims and completion counts are halved;
//   kClaimSticky: a workgroup first tries the job of its previous claim
//     (one fetch-and-add, no scan of the claim words).
// Ensembles use both (10 % faster on the finite-size-scaling mix); serving
// uses neither: its quanta end with the slowest job's chain of sweeps, which
// fewer workgroups per sweep lengthen (p50 and p99 latency rose with them).
constexpr int32_t kClaimPairs = 1, kClaimSticky = 2;
__device__ __forceinline__ int items_per_claim(int32_t nitems, int32_t flags)
{
    return (flags & kClaimPairs) && nitems >= 8 ? 2 : 1;
}

// Wave 0 looks for an open item and claims items_per_claim of them (fewer
// if the sweep has fewer left): first of job `prefer` (the job of the
// workgroup's previous claim, -1 for none) with one fetch-and-add and no
// scan, else trying jobs in priority order (order[0] first).  Returns the
// job index and writes the claimed (sweep << 32 | first item), or -1.
__device__ int find_and_claim(uint64_t *claim, const int32_t *nitems, const int32_t *order,
                              int njobs, int prefer, int32_t flags, uint64_t *got)
{
    const int lane = threadIdx.x & 63;
    if (prefer >= 0 && (flags & kClaimSticky)) {
        uint64_t w = 0;
        if (lane == 0)
            w = __hip_atomic_fetch_add(&claim[prefer],
                                       (uint64_t)items_per_claim(nitems[prefer], flags),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        w = __shfl(w, 0, 64);
        if ((uint32_t)w < (uint32_t)nitems[prefer]) {
            *got = w;
            return prefer;
        }
    }
    for (int base = 0; base < njobs; base += 64) {
        const int idx = base + lane;
        const int r = idx < njobs ? order[idx] : 0;
        bool open = false;
        if (idx < njobs) {
            const uint64_t w = ld_rlx(&claim[r]);
            open = (uint32_t)w < (uint32_t)nitems[r];
        }
        uint64_t mask = __ballot(open);
        while (mask) {
            // spread workgroups over the open jobs of this window (the
            // window holds the highest-priority jobs still open)
            uint64_t m = mask;
            for (int k = (int)(blockIdx.x % (unsigned)__popcll(mask)); k > 0; --k) m &= m - 1;
            const int pick = __ffsll((unsigned long long)m) - 1;
            const int rr = __shfl(r, pick, 64);
            uint64_t w = 0;
            if (lane == 0)
                w = __hip_atomic_fetch_add(&claim[rr], (uint64_t)items_per_claim(nitems[rr], flags),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            w = __shfl(w, 0, 64);
            if ((uint32_t)w < (uint32_t)nitems[rr]) {
                *got = w;
                return rr;
            }
            mask &= ~(1ull << pick);  // that job ran out meanwhile; try another one
        }
    }
    return -1;
}

// kCells: 0 for dead thread-cell borders, core::kDelayedCells for delayed
// ones (one kind per launch).  kGrowthOnly: every job runs p = 1, q = 0, so
// only that acceptance mode's sweep bodies are compiled in (fewer registers:
// at 1024 threads the kernel then keeps its step loops free of spills).
// budget: wall-clock ticks (wall_clock64) after which a workgroup stops
// claiming new items and exits; 0 runs until every job has finished.  An
// item once claimed is always completed, so a launch that stops early leaves
// every job at a consistent point (its open items stay claimable) and the
// next launch over the same tables continues where it stopped.
template <int kThreads, int kCells, bool kGrowthOnly>
__global__ __launch_bounds__(kThreads, kThreads / 128) void batch_kernel(const JobDesc *jobs, JobState *state,
                                                         Control *ctl, uint64_t *claim,
                                                         const int32_t *sched, int32_t njobs,
                                                         uint64_t idle_limit, uint64_t budget,
                                                         int32_t claim_flags)
{
    // static, so that the tile's base folds into the LDS instruction offsets
    __shared__ __align__(16) uint8_t smem[okpz::core::kGroupLds];
    __shared__ int s_job;     // >= 0: work; -1: exit; -2: retry
    __shared__ uint64_t s_claim;
    __shared__ int s_width;   // 1: the job just reached a sampling time
    __shared__ int64_t s_out[4];
    const int tid = threadIdx.x;
    uint64_t idle = 0, seen = 0;
    const int32_t *nitems = sched, *order = sched + njobs;
    const uint64_t t_begin = budget ? (uint64_t)wall_clock64() : 0;
    int last = -1;  // job of the previous claim (wave 0, uniform)

    while (true) {
        if (tid < 64) {
            uint64_t w = 0;
            const bool over = budget && (uint64_t)wall_clock64() - t_begin > budget;
            int r = over ? -1 : find_and_claim(claim, nitems, order, njobs, last, claim_flags, &w);
            if (r >= 0) last = r;
            if (tid == 0) {
                if (over) {
                    r = -1;
                } else if (r >= 0) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the job's state and lattice
                    idle = 0;
                } else if (__hip_atomic_load(&ctl->finished, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_SYSTEM) >= njobs ||
                           __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_SYSTEM) != 0) {
                    r = -1;
                } else {
                    // nothing open: retry after a short sleep, unless no sweep
                    // has completed anywhere for idle_limit probes
                    r = -2;
                    const uint64_t p = ld_rlx(&ctl->progress);
                    if (p != seen) {
                        seen = p;
                        idle = 0;
                    } else if (++idle > idle_limit) {
                        __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        r = -1;
                    }
                    if (r == -2) __builtin_amdgcn_s_sleep(16);
                }
                s_job = r;
                s_claim = w;
            }
        }
        __syncthreads();
        // uniform across the workgroup: readfirstlane lets the job's
        // descriptor and state be fetched with scalar loads into SGPRs
        const int r = __builtin_amdgcn_readfirstlane(s_job);
        const uint64_t w = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)s_claim);
        if (r == -1) break;
        if (r == -2) {
            __syncthreads();  // every thread has read s_job before the next claim rewrites it
            continue;
        }
        // (with an item, the group's own barriers separate these reads from the
        // next claim)

        const int item = (int)(uint32_t)w;
        const JobDesc jd = jobs[r];
        const JobState js = state[r];
        const SweepLaunch a = make_launch(jd, js);
        const int n_items = min(items_per_claim(jd.nitems, claim_flags), jd.nitems - item);
        const int g_end = min(jd.ngroups, (item + n_items) * jd.chunk);
        for (int gi = item * jd.chunk; gi < g_end; ++gi) {
            const int b0 = gi * jd.G;
            const int Gc = min(jd.G, jd.nbx * jd.nby - b0);
            if (kGrowthOnly || jd.mode == core::kGrowth)
                run_group<kThreads, core::kGrowth | kCells>(a, b0, Gc, smem);
            else if constexpr (!kGrowthOnly) {
                if (jd.mode == core::kFixed)
                    run_group<kThreads, core::kFixed | kCells>(a, b0, Gc, smem);
                else
                    run_group<kThreads, core::kDraw | kCells>(a, b0, Gc, smem);
            }
            __syncthreads();  // the group's tile is reused by the next group
        }

        if (tid == 0) {
            s_width = 0;
            // release these items' lattice words; the last item acquires
            // all (the increments form one release sequence)
            const uint32_t d = __hip_atomic_fetch_add(&state[r].done, (uint32_t)n_items,
                                                      __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) +
                               (uint32_t)n_items;
            if (d == (uint32_t)jd.nitems) {  // last item of sweep s: advance the job
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
                    publish(jd, ns, ctl, claim, r);
            }
        }
        __syncthreads();
        if (s_width) {
            const JobState ns = state[r];
            const LatticeView v{ns.cur ? jd.buf[1] : jd.buf[0], jd.Lx, jd.Ly, jd.W, ns.ox};
            const int lane = tid & 63, wave = tid >> 6, nwave = kThreads / 64;
            uint32_t *lut = reinterpret_cast<uint32_t *>(smem + 20 * 1024);
            core::width_lut_build(lut);
            __syncthreads();
            // one word per lane: the narrow form keeps the kernel's registers
            // down (a 1024 x 1024 lattice's rows are 32 words, one pass)
            for (int y = wave; y < jd.Ly; y += nwave) core::width_row<1>(v, y, lane, lut, jd.rows);
            __syncthreads();  // rows are read back by other waves of this workgroup (same CU)
            core::width_combine(jd.rows, jd.Lx, jd.Ly, s_out, reinterpret_cast<int64_t *>(smem));
            if (tid == 0) {
                int64_t *o = jd.samples + 6 * (size_t)ns.next_sample;
                o[0] = ns.s;
                o[1] = s_out[0];
                o[2] = s_out[1];
                o[3] = s_out[2];
                o[4] = s_out[3];
                o[5] = __hip_atomic_load(jd.h0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                JobState n2 = ns;
                n2.next_sample = ns.next_sample + 1;
                state[r] = n2;
                publish(jd, n2, ctl, claim, r);
            }
            __syncthreads();
        }
    }
}

// One width sample of a job run with plain sweep launches: t, the 128-bit
// sums from out[0..3] and H0, in the layout the persistent kernel writes.
__global__ void record_sample_kernel(int64_t *sample, int32_t t, const int64_t *out,
                                     const int64_t *h0)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sample[0] = t;
        for (int i = 0; i < 4; ++i) sample[1 + i] = out[i];
        sample[5] = *h0;
    }
}

// Flat zig-zag state h = (x+y) mod 2 in copy 0 of every job, H0 = 0.
__global__ void init_jobs_kernel(const JobDesc *jobs, int32_t njobs)
{
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

// Flat state in copy 0 of one job, H0 = 0.
__global__ void init_one_kernel(JobDesc jd)
{
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
    uint64_t *d_claim = nullptr;
    int32_t *d_sched = nullptr;
    int threads = 512;  // two workgroups per CU (1024 for growth-only tables, set at creation)
    int workgroups = 0;  // 0: two per compute unit
    int cus = 0;
    hipStream_t stream = nullptr;
    bool ran = false;
    bool started = false;  // okpz_batch_start done, run not yet complete
    float last_ms = 0.f;
    int32_t finished = 0;  // jobs finished in the started run
    double tick_khz = 0.0;  // wall_clock64 rate
    int32_t cell_borders = OKPZ_CELLS_DEAD;
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

// Measurement times of Sec. III as the 32-bit sweep counts the job tables
// hold (t_max < 2^31 is checked at submission).
std::vector<int32_t> sample_times(int64_t t_max, double m)
{
    const std::vector<int64_t> v = okpz::host::sample_times(t_max, m);
    return std::vector<int32_t>(v.begin(), v.end());
}

size_t al(size_t n) { return (n + 255) / 256 * 256; }

// (Re)start every job from the flat state with the given sweep limit.
// Work items of a sweep: a claim (one atomic on the job's claim word) and a
// completion count each, so a large lattice hands out its groups in chunks:
// one atomic on one word takes about a microsecond, far longer than a
// group's share of a sweep on a full device.
constexpr int kItemsPerSweep = 1024;

void set_items(JobDesc &d)
{
    d.chunk = std::max(1, (d.ngroups + kItemsPerSweep - 1) / kItemsPerSweep);
    d.nitems = (d.ngroups + d.chunk - 1) / d.chunk;
}

int reset(okpz_batch *b, const std::vector<int32_t> &tmax)
{
    const int n = (int)b->jobs.size();
    std::vector<JobState> st(n);
    std::memset(st.data(), 0, st.size() * sizeof(JobState));
    std::vector<JobDesc> desc = b->desc;
    std::vector<uint64_t> claim(n);
    // items per sweep of each job, then the scan order: most remaining work
    // first, so the longest dependency chains never wait behind short ones
    std::vector<int32_t> sched(2 * (size_t)n);
    int finished = 0;
    for (int r = 0; r < n; ++r) {
        desc[r].t_max = tmax[r];
        // sampling times beyond the limit are not reached
        int ns = 0;
        while (ns < (int)b->times[r].size() && b->times[r][ns] <= tmax[r]) ++ns;
        desc[r].nsamp = ns;
        sched[r] = desc[r].nitems;
        if (desc[r].t_max == 0) {
            claim[r] = okpz::batch::kClosed;
            ++finished;
        } else {
            claim[r] = 0;  // sweep 0, group 0
        }
    }
    std::vector<int32_t> order(n);
    for (int r = 0; r < n; ++r) order[r] = r;
    auto work = [&](int r) { return (int64_t)desc[r].Lx * desc[r].Ly * desc[r].t_max; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    std::copy(order.begin(), order.end(), sched.begin() + n);
    Control ctl{};
    ctl.finished = finished;
    BHIP(hipMemcpyAsync(b->d_desc, desc.data(), n * sizeof(JobDesc), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_state, st.data(), n * sizeof(JobState), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_claim, claim.data(), n * 8, hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_sched, sched.data(), sched.size() * 4, hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, b->stream));
    int maxwords = 0;
    for (auto &d : desc) maxwords = std::max(maxwords, 2 * d.Ly * d.W);
    const int bx = std::min(4096, (maxwords + 255) / 256);
    hipLaunchKernelGGL(okpz::batch::init_jobs_kernel, dim3(bx, n), dim3(256), 0, b->stream, b->d_desc, n);
    BHIP(hipGetLastError());
    BHIP(hipStreamSynchronize(b->stream));
    return OKPZ_OK;
}

// Device pointers of one persistent launch over a job table.
struct Ring {
    JobDesc *desc;
    JobState *state;
    Control *ctl;
    uint64_t *claim;
    int32_t *sched;  // items per sweep, then scan order
    int njobs;
    hipStream_t stream;
    int delayed_cells;  // 1: delayed thread-cell borders
    uint64_t budget = 0;  // wall-clock ticks per launch (0: run to the end)
    int32_t claim_flags = 0;  // kClaimPairs | kClaimSticky for ensembles
    int growth_only = 0;  // 1: every job runs p = 1, q = 0
};

template <int kThreads, int kCells>
hipError_t launch_ring(const Ring &R, int wgs)
{
    // about 2 s without any group completing anywhere (one probe: a scan of
    // the claim words plus a sleep of 16 x 64 cycles)
    const uint64_t idle_limit = 1ull << 19;
    if (R.growth_only)
        hipLaunchKernelGGL((okpz::batch::batch_kernel<kThreads, kCells, true>), dim3(wgs), dim3(kThreads),
                           0, R.stream, R.desc, R.state, R.ctl, R.claim, R.sched, (int32_t)R.njobs,
                           idle_limit, R.budget, R.claim_flags);
    else
        hipLaunchKernelGGL((okpz::batch::batch_kernel<kThreads, kCells, false>), dim3(wgs),
                           dim3(kThreads), 0, R.stream, R.desc, R.state, R.ctl, R.claim, R.sched,
                           (int32_t)R.njobs, idle_limit, R.budget, R.claim_flags);
    return hipGetLastError();
}

template <int kCells>
hipError_t launch_cells(const Ring &R, int threads, int wgs)
{
    switch (threads) {
    case 256: return launch_ring<256, kCells>(R, wgs);
    case 512: return launch_ring<512, kCells>(R, wgs);
    default: return launch_ring<1024, kCells>(R, wgs);
    }
}

hipError_t launch_any(const Ring &R, int threads, int wgs)
{
    if (R.delayed_cells) return launch_cells<okpz::core::kDelayedCells>(R, threads, wgs);
    return launch_cells<0>(R, threads, wgs);
}

// After a launch: OKPZ_OK if every job reached its stop target (or, for a
// launch with a time budget, if the watchdog did not fire); *finished gets
// the number of jobs that have.
int check_control(const Ring &R, int32_t *finished = nullptr)
{
    Control ctl;
    BHIP(hipMemcpy(&ctl, R.ctl, sizeof ctl, hipMemcpyDeviceToHost));
    if (finished) *finished = ctl.finished;
    if (ctl.error == 1)
        return bfail(OKPZ_EDEVICE, "persistent launch watchdog: no progress (finished %d of %d)",
                     ctl.finished, R.njobs);
    if (ctl.finished != R.njobs && R.budget == 0)
        return bfail(OKPZ_EDEVICE, "launch ended with %d of %d jobs finished", ctl.finished, R.njobs);
    return OKPZ_OK;
}

Ring ring_of(okpz_batch *b)
{
    Ring R{b->d_desc, b->d_state, b->d_ctl, b->d_claim, b->d_sched, (int)b->jobs.size(), b->stream,
           b->cell_borders == OKPZ_CELLS_DELAYED ? 1 : 0};
    R.growth_only = 1;
    for (const auto &d : b->desc) R.growth_only &= d.mode == okpz::core::kGrowth ? 1 : 0;
    return R;
}

int run(okpz_batch *b, int threads, int wgs, float *ms, uint64_t budget = 0,
        int32_t *finished = nullptr)
{
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    BHIP(hipEventRecord(e0, b->stream));
    Ring R = ring_of(b);
    R.budget = budget;
    R.claim_flags = okpz::batch::kClaimPairs | okpz::batch::kClaimSticky;
    hipError_t e = launch_any(R, threads, wgs);
    if (e != hipSuccess) return bfail(OKPZ_EDEVICE, "batch launch: %s", hipGetErrorString(e));
    BHIP(hipEventRecord(e1, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    float t = 0.f;
    BHIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms) *ms = t;
    return check_control(R, finished);
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
        set_items(d);
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
    (void)groups;
    const size_t qoff = total;
    total += al((size_t)n_jobs * 8) + al((size_t)n_jobs * 8);
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
    b->d_claim = reinterpret_cast<uint64_t *>(base + qoff);
    b->d_sched = reinterpret_cast<int32_t *>(base + qoff + al((size_t)n_jobs * 8));
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
    // an all-(1, 0) table runs the growth-only kernel, whose step loops stay
    // free of spills at 1024 threads and two workgroups per CU
    bool growth = true;
    for (const auto &d : b->desc) growth = growth && d.mode == okpz::core::kGrowth;
    if (growth) b->threads = 1024;
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

int okpz_batch_set_cell_borders(okpz_batch *b, int32_t kind)
{
    if (!b) return bfail(OKPZ_EINVAL, "null handle");
    if (kind != OKPZ_CELLS_DEAD && kind != OKPZ_CELLS_DELAYED)
        return bfail(OKPZ_EINVAL, "cell border kind %d is neither dead (0) nor delayed (1)", kind);
    b->cell_borders = kind;
    return OKPZ_OK;
}

int okpz_batch_get_cell_borders(const okpz_batch *b, int32_t *kind)
{
    if (!b || !kind) return bfail(OKPZ_EINVAL, "null argument");
    *kind = b->cell_borders;
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
    int rc = okpz_batch_start(b);
    if (rc != OKPZ_OK) return rc;
    const int wgs = b->workgroups ? b->workgroups : 2 * b->cus;
    rc = run(b, b->threads, wgs, &b->last_ms);
    b->started = false;
    if (rc == OKPZ_OK) b->ran = true;
    return rc;
}

int okpz_batch_start(okpz_batch *b)
{
    if (!b) return bfail(OKPZ_EINVAL, "null batch");
    std::vector<int32_t> tmax(b->jobs.size());
    for (size_t r = 0; r < b->jobs.size(); ++r) tmax[r] = (int32_t)b->jobs[r].t_max;
    int rc = reset(b, tmax);
    if (rc != OKPZ_OK) return rc;
    b->ran = false;
    b->started = true;
    b->last_ms = 0.f;
    b->finished = 0;
    return OKPZ_OK;
}

int okpz_batch_run_for(okpz_batch *b, double max_ms, int32_t *finished)
{
    if (!b) return bfail(OKPZ_EINVAL, "null batch");
    if (!b->started) return bfail(OKPZ_EINVAL, "okpz_batch_start has not been called");
    if (!(max_ms > 0.0) || max_ms > 3.6e6) return bfail(OKPZ_EINVAL, "max_ms must lie in (0, 3.6e6]");
    if (b->tick_khz <= 0.0) {
        int dev = 0, khz = 0;
        BHIP(hipGetDevice(&dev));
        BHIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        if (khz <= 0) return bfail(OKPZ_EDEVICE, "device reports no wall-clock rate");
        b->tick_khz = khz;
    }
    const uint64_t budget = std::max<uint64_t>(1, (uint64_t)(max_ms * b->tick_khz));
    const int wgs = b->workgroups ? b->workgroups : 2 * b->cus;
    float ms = 0.f;
    int32_t done = 0;
    int rc = run(b, b->threads, wgs, &ms, budget, &done);
    b->last_ms += ms;
    if (rc != OKPZ_OK) {
        b->started = false;
        return rc;
    }
    b->finished = done;
    if (finished) *finished = done;
    if (done == (int32_t)b->jobs.size()) {
        b->started = false;
        b->ran = true;
    }
    return OKPZ_OK;
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
    // a scaled-down copy of the workload: the same mix of short and long
    // dependency chains, the longest job running trial_mcs sweeps
    int64_t longest = 1;
    for (const auto &j : b->jobs) longest = std::max<int64_t>(longest, j.t_max);
    std::vector<int32_t> tmax(b->jobs.size());
    for (size_t r = 0; r < b->jobs.size(); ++r) {
        const int64_t t = b->jobs[r].t_max;
        const int64_t scaled = (t * std::min<int64_t>(trial_mcs, longest) + longest - 1) / longest;
        tmax[r] = (int32_t)(t == 0 ? 0 : std::max<int64_t>(1, std::min<int64_t>(t, scaled)));
    }
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
    b->started = false;
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

}  // extern "C"

namespace {

// W^2 = (N S2 - S1^2) / N^2 (Eq. (Wdef)) of every sample with t >= t_from of
// every job of size Lx x Ly, from the exact integer numerator.
int w2_values(okpz_batch *b, int64_t Lx, int64_t Ly, int64_t t_from, std::vector<double> *out)
{
    out->clear();
    for (int32_t r = 0; r < (int32_t)b->jobs.size(); ++r) {
        if (b->jobs[r].Lx != Lx || b->jobs[r].Ly != Ly) continue;
        int32_t n = 0;
        int rc = okpz_batch_samples(b, r, nullptr, nullptr, nullptr, 0, &n);
        if (rc != OKPZ_OK) return rc;
        std::vector<int64_t> t(n), s1(n), s2(n);
        rc = okpz_batch_samples(b, r, t.data(), s1.data(), s2.data(), n, &n);
        if (rc != OKPZ_OK) return rc;
        const __int128 N = (__int128)Lx * Ly;
        for (int i = 0; i < n; ++i) {
            if (t[i] < t_from) continue;
            const __int128 num = N * (__int128)s2[i] - (__int128)s1[i] * s1[i];
            out->push_back((double)num / ((double)N * (double)N));
        }
    }
    return OKPZ_OK;
}

}  // namespace

extern "C" {

int okpz_batch_w2_histogram(okpz_batch *b, int64_t Lx, int64_t Ly, int64_t t_from, double lo,
                            double hi, int32_t nbins, int64_t *counts, int64_t *under, int64_t *over)
{
    if (!b || !counts) return bfail(OKPZ_EINVAL, "null argument");
    if (nbins <= 0 || !(hi > lo)) return bfail(OKPZ_EINVAL, "need nbins > 0 and hi > lo");
    std::vector<double> w;
    int rc = w2_values(b, Lx, Ly, t_from, &w);
    if (rc != OKPZ_OK) return rc;
    for (int i = 0; i < nbins; ++i) counts[i] = 0;
    int64_t u = 0, o = 0;
    for (double w2 : w) {
        const double f = (w2 - lo) / (hi - lo) * nbins;
        if (f < 0) ++u;
        else if (f >= nbins) ++o;
        else ++counts[(int)f];
    }
    if (under) *under = u;
    if (over) *over = o;
    return OKPZ_OK;
}

int okpz_batch_w2_cumulants(okpz_batch *b, int64_t Lx, int64_t Ly, int64_t t_from, int64_t *count,
                            double *nu, double *kappa)
{
    if (!b || !count || !nu || !kappa) return bfail(OKPZ_EINVAL, "null argument");
    std::vector<double> w;
    int rc = w2_values(b, Lx, Ly, t_from, &w);
    if (rc != OKPZ_OK) return rc;
    *count = (int64_t)w.size();
    if (w.empty()) return bfail(OKPZ_EINVAL, "no samples of size %lldx%lld at t >= %lld",
                                (long long)Lx, (long long)Ly, (long long)t_from);
    long double m[5] = {0, 0, 0, 0, 0};
    for (double v : w) {
        const long double x = v;
        m[1] += x;
        m[2] += x * x;
        m[3] += x * x * x;
        m[4] += x * x * x * x;
    }
    for (int n = 1; n <= 4; ++n) m[n] /= (long double)w.size();
    // cumulants from the non-central moments (Sec. IV, Eq. (cumulants))
    const long double k1 = m[1];
    const long double k2 = m[2] - m[1] * m[1];
    const long double k3 = m[3] - 3 * m[1] * m[2] + 2 * m[1] * m[1] * m[1];
    const long double k4 = m[4] - 4 * m[3] * m[1] - 3 * m[2] * m[2] + 12 * m[1] * m[1] * m[2] -
                           6 * m[1] * m[1] * m[1] * m[1];
    for (int n = 0; n < 4; ++n) nu[n] = (double)m[n + 1];
    kappa[0] = (double)k1;
    kappa[1] = (double)k2;
    kappa[2] = (double)k3;
    kappa[3] = (double)k4;
    return OKPZ_OK;
}

int okpz_batch_psi(okpz_batch *b, int64_t Lx, int64_t Ly, int64_t t_from, double x_hi,
                   int32_t nbins, double *psi, int64_t *count)
{
    if (!b || !psi || !count) return bfail(OKPZ_EINVAL, "null argument");
    if (nbins <= 0 || !(x_hi > 0)) return bfail(OKPZ_EINVAL, "need nbins > 0 and x_hi > 0");
    std::vector<double> w;
    int rc = w2_values(b, Lx, Ly, t_from, &w);
    if (rc != OKPZ_OK) return rc;
    *count = (int64_t)w.size();
    if (w.empty()) return bfail(OKPZ_EINVAL, "no samples of size %lldx%lld at t >= %lld",
                                (long long)Lx, (long long)Ly, (long long)t_from);
    long double mean = 0;
    for (double v : w) mean += v;
    mean /= (long double)w.size();
    if (!(mean > 0)) return bfail(OKPZ_EINVAL, "mean W^2 is not positive");
    for (int i = 0; i < nbins; ++i) psi[i] = 0;
    const double dx = x_hi / nbins;
    for (double v : w) {
        const double f = (double)((long double)v / mean) / dx;
        if (f >= 0 && f < nbins) psi[(int)f] += 1.0;
    }
    // density of x = W^2 / <W^2>: Psi_L(x) = <W^2> P_L(W^2) (Sec. IV)
    for (int i = 0; i < nbins; ++i) psi[i] /= (double)w.size() * dx;
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


// ===========================================================================
// Serving: continuous batching of simulation jobs
// ===========================================================================
//
// Jobs are submitted with an arrival time.  Each call to okpz_serve_step is
// one quantum: jobs whose arrival time has passed are admitted in arrival
// order while a slot is free and their device bytes fit the HBM budget (their
// lattices are allocated and stay resident until they finish); then one
// persistent launch advances every resident job by its quantum share of
// sweeps, all jobs' groups interleaved on the device; finished jobs are
// retired (samples copied out, memory freed) and their latency recorded.
//
// Shares: a quantum lasts about T = quantum_sites / kNominalRate seconds.
// The sweeps of one job form a sequential chain, each taking about
// kSweepLatency + L^2 / kNominalRate seconds (a small lattice is latency
// bound, a large one throughput bound), so a job's share is the number of
// sweeps its chain completes in T (at least one).  Large jobs then keep the
// device busy while small jobs' chains run beside them, and no small job
// stretches the quantum.  A job's results do not depend on when it ran or
// with which other jobs.
#include <chrono>
#include <deque>

namespace {

struct ServeJob {
    okpz_job job{};
    double arrival = 0, admit = -1, finish = -1;
    int state = 0;  // 0 waiting, 1 running, 2 done, 3 cancelled
    int slot = -1;
    bool keep_lattice = false;
    size_t bytes = 0;
    void *mem = nullptr;
    JobDesc desc{};
    std::vector<int32_t> times;
    int32_t s = 0;  // MCS completed (host mirror)
    // large lattices run as plain per-lattice sweeps (see okpz_serve_step);
    // their state lives on the host
    bool grid = false;
    int32_t ox = 0, cur = 0, next_sample = 0;
    std::vector<int64_t> raw;
    std::vector<uint8_t> lattice;
    int64_t h0 = 0;
};

size_t job_bytes(const okpz_job &j, size_t nsamp)
{
    const size_t lat = al(2 * (size_t)j.Ly * (size_t)(j.Lx / 32) * 4);
    return 2 * lat + al(8) + al((okpz::width_scratch_words(j.Ly) + 4) * 8) +
           al(6 * 8 * std::max<size_t>(1, nsamp)) +
           al(4 * std::max<size_t>(1, nsamp));
}

}  // namespace

// Device model behind the quantum shares: site updates per second of the
// whole device on one large lattice, and the time of one sweep of a lattice
// that fits one workgroup (staging, 64 barrier-separated steps, store and
// the hand-over to the next sweep).
constexpr double kNominalRate = 1.0e12;
// Lattices with at least this many groups per sweep (4096 x 4096 and up)
// run as plain per-lattice sweep launches on a second stream, next to the
// persistent launch: one large sweep fills the device by itself, while
// through the claim words its groups would be handed out one atomic at a
// time.
constexpr int kGridGroups = 256;
constexpr double kSweepLatency = 2.0e-5;

struct okpz_server {
    size_t budget = 0, used = 0;
    int max_slots = 0;
    int64_t quantum_sites = 0;
    double m = 0.01;
    std::vector<ServeJob> jobs;
    std::deque<int64_t> waiting;  // sorted by arrival
    std::vector<int64_t> slot_job;
    void *mem = nullptr;
    JobDesc *d_desc = nullptr;
    JobState *d_state = nullptr;
    Control *d_ctl = nullptr;
    uint64_t *d_claim = nullptr;
    int32_t *d_sched = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t grid_stream = nullptr;  // plain sweeps of large lattices
    int threads = 512, wgs = 0, cus = 0;  // two workgroups per CU without spills
    int32_t cell_borders = OKPZ_CELLS_DEAD;  // for every job of the server
    std::chrono::steady_clock::time_point t0;
    int64_t quanta = 0, done = 0;
    double device_ms = 0;
};

namespace {

double now_s(const okpz_server *s)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

// Retire a resident job: copy its samples (the first `nsamp` of them; all for
// a finished job), H0 and, on request, its lattice to the host, free its
// memory and its slot.  Called between quanta only (no device work of the
// server is in flight then).
int retire(okpz_server *sv, ServeJob &J, double t, bool cancelled = false)
{
    const JobDesc &d = J.desc;
    int32_t nsamp = d.nsamp;
    if (cancelled) {
        if (J.grid) {
            nsamp = J.next_sample;
        } else {
            JobState st;
            BHIP(hipMemcpy(&st, sv->d_state + J.slot, sizeof st, hipMemcpyDeviceToHost));
            nsamp = st.next_sample;
        }
    }
    J.raw.assign(6 * (size_t)nsamp, 0);
    if (nsamp)
        BHIP(hipMemcpy(J.raw.data(), d.samples, 6 * 8 * (size_t)nsamp, hipMemcpyDeviceToHost));
    BHIP(hipMemcpy(&J.h0, d.h0, 8, hipMemcpyDeviceToHost));
    if (J.keep_lattice) {
        JobState st;
        BHIP(hipMemcpy(&st, sv->d_state + J.slot, sizeof st, hipMemcpyDeviceToHost));
        if (J.grid) {
            st.ox = J.ox;
            st.cur = J.cur;
        }
        std::vector<uint32_t> pl(2 * (size_t)d.Ly * d.W);
        BHIP(hipMemcpy(pl.data(), st.cur ? d.buf[1] : d.buf[0], pl.size() * 4, hipMemcpyDeviceToHost));
        J.lattice.resize((size_t)d.Lx * d.Ly);
        for (int64_t y = 0; y < d.Ly; ++y)
            for (int64_t x = 0; x < d.Lx; ++x) {
                const int64_t c = ((x - st.ox) % d.Lx + d.Lx) % d.Lx;
                const uint32_t bx = (pl[(size_t)y * d.W + (c >> 5)] >> (c & 31)) & 1u;
                const uint32_t by = (pl[((size_t)d.Ly + y) * d.W + (c >> 5)] >> (c & 31)) & 1u;
                J.lattice[y * d.Lx + x] = (uint8_t)(bx | (by << 1));
            }
    }
    BHIP(hipFree(J.mem));
    J.mem = nullptr;
    sv->used -= J.bytes;
    sv->slot_job[J.slot] = -1;
    J.slot = -1;
    J.state = cancelled ? 3 : 2;
    J.finish = t;
    if (!cancelled) ++sv->done;
    return OKPZ_OK;
}

int admit(okpz_server *sv, ServeJob &J, int slot, double t)
{
    const okpz_job &j = J.job;
    J.bytes = job_bytes(j, J.times.size());
    hipError_t e = hipMalloc(&J.mem, J.bytes);
    if (e != hipSuccess) return bfail(OKPZ_ENOMEM, "hipMalloc(%zu): %s", J.bytes, hipGetErrorString(e));
    okpz::Geometry g;
    okpz::geometry_of(j.Lx, j.Ly, &g);
    JobDesc &d = J.desc;
    std::memset(&d, 0, sizeof d);
    d.Lx = (int32_t)j.Lx;
    d.Ly = (int32_t)j.Ly;
    d.W = (int32_t)(j.Lx / 32);
    d.Bx = g.Bx;
    d.By = g.By;
    d.nbx = (int32_t)(j.Lx / g.Bx);
    d.nby = (int32_t)(j.Ly / g.By);
    d.G = okpz::core::group_size(g.Bx, g.By, d.nbx * d.nby);
    d.ngroups = (d.nbx * d.nby + d.G - 1) / d.G;
    set_items(d);
    d.k0 = (uint32_t)(j.seed & 0xffffffffu);
    d.k1 = (uint32_t)(j.seed >> 32);
    d.Tp = okpz::threshold_of(j.p);
    d.Tq = okpz::threshold_of(j.q);
    const uint64_t one = uint64_t(1) << 32;
    const bool trivial = (d.Tp == 0 || d.Tp == one) && (d.Tq == 0 || d.Tq == one);
    d.mode = !trivial ? okpz::core::kDraw
                      : (d.Tp == one && d.Tq == 0 ? okpz::core::kGrowth : okpz::core::kFixed);
    d.t_max = (int32_t)j.t_max;
    d.nsamp = (int32_t)J.times.size();
    char *p = static_cast<char *>(J.mem);
    const size_t lat = al(2 * (size_t)j.Ly * (size_t)(j.Lx / 32) * 4);
    d.buf[0] = reinterpret_cast<uint32_t *>(p);
    d.buf[1] = reinterpret_cast<uint32_t *>(p + lat);
    d.h0 = reinterpret_cast<int64_t *>(p + 2 * lat);
    d.rows = reinterpret_cast<int64_t *>(p + 2 * lat + al(8));
    const size_t rows_b = al((okpz::width_scratch_words(j.Ly) + 4) * 8);
    d.samples = reinterpret_cast<int64_t *>(p + 2 * lat + al(8) + rows_b);
    int32_t *tt = reinterpret_cast<int32_t *>(p + 2 * lat + al(8) + rows_b +
                                               al(6 * 8 * std::max<size_t>(1, d.nsamp)));
    d.sample_t = tt;
    if (d.nsamp) BHIP(hipMemcpy(tt, J.times.data(), 4 * (size_t)d.nsamp, hipMemcpyHostToDevice));
    const int bx = (int)std::min<size_t>(4096, (2 * (size_t)d.Ly * d.W + 255) / 256);
    hipLaunchKernelGGL(okpz::batch::init_one_kernel, dim3(bx), dim3(256), 0, sv->stream, d);
    BHIP(hipGetLastError());
    JobState st;
    std::memset(&st, 0, sizeof st);
    BHIP(hipMemcpyAsync(sv->d_state + slot, &st, sizeof st, hipMemcpyHostToDevice, sv->stream));
    BHIP(hipStreamSynchronize(sv->stream));
    sv->used += J.bytes;
    sv->slot_job[slot] = (int64_t)(&J - sv->jobs.data());
    J.slot = slot;
    J.state = 1;
    J.admit = t;
    J.s = 0;
    J.grid = d.ngroups >= kGridGroups;
    J.ox = 0;
    J.cur = 0;
    J.next_sample = 0;
    return OKPZ_OK;
}

// Advance a large job to sweep `stop` with plain per-lattice sweep launches
// (and width launches at its sampling times) on the server's second stream.
int run_grid(okpz_server *sv, ServeJob &J, int64_t stop)
{
    const JobDesc &d = J.desc;
    okpz::Geometry g;
    okpz::geometry_of(d.Lx, d.Ly, &g);
    okpz::SweepLaunch a{};
    a.h0 = d.h0;
    a.Lx = d.Lx;
    a.Ly = d.Ly;
    a.W = d.W;
    a.Bx = d.Bx;
    a.By = d.By;
    a.nbx = d.nbx;
    a.nby = d.nby;
    a.k0 = d.k0;
    a.k1 = d.k1;
    a.Tp = d.Tp;
    a.Tq = d.Tq;
    a.need_accept_draws = d.mode == okpz::core::kDraw ? 1 : 0;
    a.delayed_cells = sv->cell_borders == OKPZ_CELLS_DELAYED ? 1 : 0;
    while (J.s < stop) {
        const uint32_t sw = (uint32_t)J.s;
        int32_t sx, sy;
        okpz::block_shift(d.k0, d.k1, sw, g, &sx, &sy);
        const int64_t x00 = (d.Lx - sx) % d.Lx, y00 = (d.Ly - sy) % d.Ly;
        a.blk00 = (int32_t)((y00 / d.By) * d.nbx + x00 / d.Bx);
        a.u00 = (int32_t)(x00 % d.Bx);
        a.v00 = (int32_t)(y00 % d.By);
        a.src = d.buf[J.cur];
        a.dst = d.buf[J.cur ^ 1];
        a.ox_src = J.ox;
        a.sx = sx;
        a.sy = sy;
        a.s = sw;
        hipError_t e = okpz::launch_sweep(a, 1024, sv->grid_stream);
        if (e != hipSuccess) return bfail(OKPZ_EDEVICE, "serve sweep: %s", hipGetErrorString(e));
        J.cur ^= 1;
        J.ox = sx;
        J.s += 1;
        if (J.next_sample < d.nsamp && J.times[J.next_sample] == J.s) {
            const okpz::LatticeView v{d.buf[J.cur], d.Lx, d.Ly, d.W, J.ox};
            int64_t *out = d.rows + okpz::width_scratch_words(d.Ly);
            e = okpz::launch_width(v, d.rows, out, sv->grid_stream);
            if (e != hipSuccess) return bfail(OKPZ_EDEVICE, "serve width: %s", hipGetErrorString(e));
            hipLaunchKernelGGL(okpz::batch::record_sample_kernel, dim3(1), dim3(64), 0,
                               sv->grid_stream, d.samples + 6 * (size_t)J.next_sample, J.s, out,
                               d.h0);
            BHIP(hipGetLastError());
            ++J.next_sample;
        }
    }
    return OKPZ_OK;
}

}  // namespace

extern "C" {

int okpz_serve_create(okpz_server **out, size_t hbm_budget, int32_t max_slots,
                      int64_t quantum_sites, double m)
{
    if (!out) return bfail(OKPZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots <= 0 || max_slots > 4096) return bfail(OKPZ_EINVAL, "max_slots must be in [1, 4096]");
    if (quantum_sites <= 0) return bfail(OKPZ_EINVAL, "quantum_sites must be positive");
    if (!(m > 0.0) || m > 10.0) return bfail(OKPZ_EINVAL, "sampling exponent m must be in (0, 10]");
    if (hbm_budget == 0) return bfail(OKPZ_EINVAL, "hbm_budget must be positive");
    okpz_server *sv = new okpz_server();
    sv->budget = hbm_budget;
    sv->max_slots = max_slots;
    sv->quantum_sites = quantum_sites;
    sv->m = m;
    sv->slot_job.assign(max_slots, -1);
    const size_t total = al(max_slots * sizeof(JobDesc)) + al(max_slots * sizeof(JobState)) +
                         al(sizeof(Control)) + al((size_t)max_slots * 8) + al((size_t)max_slots * 8);
    hipError_t e = hipMalloc(&sv->mem, total);
    if (e != hipSuccess) {
        delete sv;
        return bfail(OKPZ_ENOMEM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
    }
    char *base = static_cast<char *>(sv->mem);
    sv->d_desc = reinterpret_cast<JobDesc *>(base);
    base += al(max_slots * sizeof(JobDesc));
    sv->d_state = reinterpret_cast<JobState *>(base);
    base += al(max_slots * sizeof(JobState));
    sv->d_ctl = reinterpret_cast<Control *>(base);
    base += al(sizeof(Control));
    sv->d_claim = reinterpret_cast<uint64_t *>(base);
    sv->d_sched = reinterpret_cast<int32_t *>(base + al((size_t)max_slots * 8));
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&sv->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (sv->cus <= 0) sv->cus = 256;
    e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->grid_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (sv->stream) (void)hipStreamDestroy(sv->stream);
        (void)hipFree(sv->mem);
        delete sv;
        return bfail(OKPZ_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    sv->t0 = std::chrono::steady_clock::now();
    *out = sv;
    return OKPZ_OK;
}

int okpz_serve_set_mapping(okpz_server *sv, int32_t threads, int32_t workgroups)
{
    if (!sv) return bfail(OKPZ_EINVAL, "null server");
    if (threads != 256 && threads != 512 && threads != 1024)
        return bfail(OKPZ_EINVAL, "threads per workgroup must be 256, 512 or 1024");
    if (workgroups < 0 || workgroups > (1 << 16)) return bfail(OKPZ_EINVAL, "workgroups out of range");
    sv->threads = threads;
    sv->wgs = workgroups;
    return OKPZ_OK;
}

int okpz_serve_set_cell_borders(okpz_server *sv, int32_t kind)
{
    if (!sv) return bfail(OKPZ_EINVAL, "null server");
    if (kind != OKPZ_CELLS_DEAD && kind != OKPZ_CELLS_DELAYED)
        return bfail(OKPZ_EINVAL, "cell border kind %d is neither dead (0) nor delayed (1)", kind);
    if (!sv->jobs.empty()) return bfail(OKPZ_EINVAL, "cell borders are set before the first submit");
    sv->cell_borders = kind;
    return OKPZ_OK;
}

int okpz_serve_get_cell_borders(const okpz_server *sv, int32_t *kind)
{
    if (!sv || !kind) return bfail(OKPZ_EINVAL, "null argument");
    *kind = sv->cell_borders;
    return OKPZ_OK;
}

int okpz_serve_now(okpz_server *sv, double *now)
{
    if (!sv || !now) return bfail(OKPZ_EINVAL, "null argument");
    *now = now_s(sv);
    return OKPZ_OK;
}

int okpz_serve_submit(okpz_server *sv, const okpz_job *job, double arrival_s, int32_t keep_lattice,
                      int64_t *id)
{
    if (!sv || !job || !id) return bfail(OKPZ_EINVAL, "null argument");
    const okpz_job &j = *job;
    if (!side_ok(j.Lx) || !side_ok(j.Ly))
        return bfail(OKPZ_EINVAL, "sides must be multiples of 32 in [32, 8192]");
    if (!(j.p >= 0.0 && j.p <= 1.0) || !(j.q >= 0.0 && j.q <= 1.0))
        return bfail(OKPZ_EINVAL, "p and q must lie in [0,1]");
    if (j.t_max < 0 || j.t_max >= (int64_t(1) << 31)) return bfail(OKPZ_EINVAL, "t_max out of range");
    ServeJob J;
    J.job = j;
    J.arrival = arrival_s < 0 ? now_s(sv) : arrival_s;
    J.keep_lattice = keep_lattice != 0;
    J.times = sample_times(j.t_max, sv->m);
    if (job_bytes(j, J.times.size()) > sv->budget)
        return bfail(OKPZ_EBUSY, "job needs %zu bytes, more than the whole budget",
                     job_bytes(j, J.times.size()));
    sv->jobs.push_back(std::move(J));
    const int64_t k = (int64_t)sv->jobs.size() - 1;
    // keep the waiting list in arrival order (stable)
    auto it = sv->waiting.end();
    while (it != sv->waiting.begin() && sv->jobs[*(it - 1)].arrival > sv->jobs[k].arrival) --it;
    sv->waiting.insert(it, k);
    *id = k;
    return OKPZ_OK;
}

int okpz_serve_step(okpz_server *sv, int32_t *running, int32_t *waiting)
{
    if (!sv) return bfail(OKPZ_EINVAL, "null server");
    double t = now_s(sv);
    // 1. admission: arrival order, a free slot and the bytes must fit
    while (!sv->waiting.empty()) {
        ServeJob &J = sv->jobs[sv->waiting.front()];
        if (J.arrival > t) break;
        int slot = -1;
        for (int i = 0; i < sv->max_slots; ++i)
            if (sv->slot_job[i] < 0) {
                slot = i;
                break;
            }
        if (slot < 0 || sv->used + job_bytes(J.job, J.times.size()) > sv->budget) break;
        int rc = admit(sv, J, slot, t);
        if (rc != OKPZ_OK) return rc;
        sv->waiting.pop_front();
        if (J.job.t_max == 0) {
            rc = retire(sv, J, now_s(sv));
            if (rc != OKPZ_OK) return rc;
        }
    }
    // 2. quantum: every resident job advances by its share; small jobs in one
    // persistent launch, large ones (J.grid) as plain sweep launches on the
    // second stream at the same time
    std::vector<JobDesc> desc(sv->max_slots);
    std::vector<uint64_t> claim(sv->max_slots, okpz::batch::kClosed);
    // items per sweep of each slot, then the scan order: oldest job first
    std::vector<int32_t> sched(2 * (size_t)sv->max_slots, 0);
    std::vector<std::pair<int64_t, int64_t>> grid_jobs;  // (job, stop)
    int active = 0, finished = 0, n_small = 0;
    for (int i = 0; i < sv->max_slots; ++i) {
        std::memset(&desc[i], 0, sizeof(JobDesc));
        const int64_t k = sv->slot_job[i];
        if (k < 0) {
            ++finished;
            continue;
        }
        ServeJob &J = sv->jobs[k];
        const double quantum_s = (double)sv->quantum_sites / kNominalRate;
        const double sweep_s = kSweepLatency + (double)(J.job.Lx * J.job.Ly) / kNominalRate;
        const int64_t share = std::max<int64_t>(1, (int64_t)(quantum_s / sweep_s));
        const int64_t stop = std::min<int64_t>(J.job.t_max, J.s + share);
        ++active;
        if (J.grid) {
            grid_jobs.push_back({k, stop});
            ++finished;  // not in the persistent launch
            continue;
        }
        desc[i] = J.desc;
        desc[i].t_max = (int32_t)stop;
        claim[i] = (uint64_t)J.s << 32;
        sched[i] = J.desc.nitems;
        ++n_small;
    }
    {
        std::vector<int32_t> order(sv->max_slots);
        for (int i = 0; i < sv->max_slots; ++i) order[i] = i;
        auto arrival = [&](int i) {
            return sv->slot_job[i] < 0 ? 1e300 : sv->jobs[sv->slot_job[i]].arrival;
        };
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return arrival(x) < arrival(y); });
        std::copy(order.begin(), order.end(), sched.begin() + sv->max_slots);
    }
    if (running) *running = active;
    if (waiting) *waiting = (int32_t)sv->waiting.size();
    if (active == 0) return OKPZ_OK;
    hipEvent_t e0, e1, eg;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    BHIP(hipEventCreate(&eg));
    BHIP(hipEventRecord(e0, sv->stream));
    const Ring R{sv->d_desc, sv->d_state, sv->d_ctl, sv->d_claim, sv->d_sched, sv->max_slots,
                 sv->stream, sv->cell_borders == OKPZ_CELLS_DELAYED ? 1 : 0};
    if (n_small > 0) {
        Control ctl{};
        ctl.finished = finished;
        BHIP(hipMemcpyAsync(sv->d_desc, desc.data(), desc.size() * sizeof(JobDesc),
                            hipMemcpyHostToDevice, sv->stream));
        BHIP(hipMemcpyAsync(sv->d_claim, claim.data(), claim.size() * 8, hipMemcpyHostToDevice,
                            sv->stream));
        BHIP(hipMemcpyAsync(sv->d_sched, sched.data(), sched.size() * 4, hipMemcpyHostToDevice,
                            sv->stream));
        BHIP(hipMemcpyAsync(sv->d_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, sv->stream));
        // beside plain sweeps, one persistent workgroup per CU leaves room for them
        const int wgs = sv->wgs ? sv->wgs : (grid_jobs.empty() ? 2 : 1) * sv->cus;
        hipError_t e = launch_any(R, sv->threads, wgs);
        if (e != hipSuccess) return bfail(OKPZ_EDEVICE, "serve launch: %s", hipGetErrorString(e));
    }
    if (!grid_jobs.empty()) {
        BHIP(hipStreamWaitEvent(sv->grid_stream, e0, 0));
        for (const auto &gj : grid_jobs) {
            const int rc = run_grid(sv, sv->jobs[gj.first], gj.second);
            if (rc != OKPZ_OK) return rc;
        }
        BHIP(hipEventRecord(eg, sv->grid_stream));
        BHIP(hipStreamWaitEvent(sv->stream, eg, 0));
    }
    BHIP(hipEventRecord(e1, sv->stream));
    BHIP(hipStreamSynchronize(sv->stream));
    float ms = 0.f;
    BHIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(eg);
    sv->device_ms += ms;
    ++sv->quanta;
    int rc = n_small > 0 ? check_control(R) : OKPZ_OK;
    if (rc != OKPZ_OK) return rc;
    // 3. retire finished jobs
    std::vector<JobState> st(sv->max_slots);
    BHIP(hipMemcpy(st.data(), sv->d_state, st.size() * sizeof(JobState), hipMemcpyDeviceToHost));
    t = now_s(sv);
    for (int i = 0; i < sv->max_slots; ++i) {
        const int64_t k = sv->slot_job[i];
        if (k < 0) continue;
        ServeJob &J = sv->jobs[k];
        if (!J.grid) J.s = st[i].s;  // grid jobs keep their state on the host
        if (J.s >= J.job.t_max) {
            rc = retire(sv, J, t);
            if (rc != OKPZ_OK) return rc;
        }
    }
    if (running) {
        int n = 0;
        for (int i = 0; i < sv->max_slots; ++i) n += sv->slot_job[i] >= 0;
        *running = n;
    }
    return OKPZ_OK;
}

int okpz_serve_job(okpz_server *sv, int64_t id, int32_t *state, double *arrival, double *admit_t,
                   double *finish)
{
    if (!sv) return bfail(OKPZ_EINVAL, "null server");
    if (id < 0 || id >= (int64_t)sv->jobs.size()) return bfail(OKPZ_EINVAL, "unknown job");
    const ServeJob &J = sv->jobs[id];
    if (state) *state = J.state;
    if (arrival) *arrival = J.arrival;
    if (admit_t) *admit_t = J.admit;
    if (finish) *finish = J.finish;
    return OKPZ_OK;
}

int okpz_serve_cancel(okpz_server *sv, int64_t id)
{
    if (!sv) return bfail(OKPZ_EINVAL, "null server");
    if (id < 0 || id >= (int64_t)sv->jobs.size()) return bfail(OKPZ_EINVAL, "unknown job");
    ServeJob &J = sv->jobs[id];
    const double t = now_s(sv);
    if (J.state == 0) {
        for (auto it = sv->waiting.begin(); it != sv->waiting.end(); ++it)
            if (*it == id) {
                sv->waiting.erase(it);
                break;
            }
        J.raw.clear();
        J.state = 3;
        J.finish = t;
        return OKPZ_OK;
    }
    if (J.state == 1) return retire(sv, J, t, true);
    return bfail(OKPZ_EINVAL, "job %lld has already %s", (long long)id,
                 J.state == 2 ? "finished" : "been cancelled");
}

int okpz_serve_samples(okpz_server *sv, int64_t id, int64_t *t, int64_t *sum_h, int64_t *sum_h2,
                       int32_t cap, int32_t *count)
{
    if (!sv || !count) return bfail(OKPZ_EINVAL, "null argument");
    if (id < 0 || id >= (int64_t)sv->jobs.size()) return bfail(OKPZ_EINVAL, "unknown job");
    const ServeJob &J = sv->jobs[id];
    if (J.state != 2 && J.state != 3)
        return bfail(OKPZ_EINVAL, "job %lld has not finished", (long long)id);
    const int n = J.state == 2 ? (int)J.times.size() : (int)(J.raw.size() / 6);
    *count = n;
    if (!t && !sum_h && !sum_h2) return OKPZ_OK;
    if (cap < n) return bfail(OKPZ_EINVAL, "capacity %d < %d samples", cap, n);
    const __int128 N = (__int128)J.job.Lx * J.job.Ly;
    const __int128 lim = (__int128)1 << 63;
    for (int i = 0; i < n; ++i) {
        const int64_t *o = &J.raw[6 * (size_t)i];
        const __int128 s1r = (__int128)(((unsigned __int128)(uint64_t)o[2] << 64) | (uint64_t)o[1]);
        const __int128 s2r = (__int128)(((unsigned __int128)(uint64_t)o[4] << 64) | (uint64_t)o[3]);
        const __int128 H0 = o[5];
        const __int128 S1 = s1r + N * H0;
        const __int128 S2 = s2r + 2 * H0 * s1r + N * H0 * H0;
        if (S1 >= lim || S1 < -lim || S2 >= lim || S2 < 0)
            return bfail(OKPZ_EOVERFLOW, "job %lld sample %d exceeds int64", (long long)id, i);
        if (t) t[i] = o[0];
        if (sum_h) sum_h[i] = (int64_t)S1;
        if (sum_h2) sum_h2[i] = (int64_t)S2;
    }
    return OKPZ_OK;
}

int okpz_serve_result(okpz_server *sv, int64_t id, uint8_t *host, size_t bytes, int64_t *h0)
{
    if (!sv) return bfail(OKPZ_EINVAL, "null server");
    if (id < 0 || id >= (int64_t)sv->jobs.size()) return bfail(OKPZ_EINVAL, "unknown job");
    const ServeJob &J = sv->jobs[id];
    if (J.state != 2 && !(J.state == 3 && J.admit >= 0))
        return bfail(OKPZ_EINVAL, "job %lld has not finished (or was cancelled before it ran)",
                     (long long)id);
    if (h0) *h0 = J.h0;
    if (host) {
        if (!J.keep_lattice) return bfail(OKPZ_EINVAL, "job %lld did not keep its lattice", (long long)id);
        if (bytes < J.lattice.size()) return bfail(OKPZ_EINVAL, "host buffer too small");
        std::memcpy(host, J.lattice.data(), J.lattice.size());
    }
    return OKPZ_OK;
}

int okpz_serve_stats(okpz_server *sv, int64_t *quanta, double *device_ms, int64_t *done,
                     size_t *bytes_in_use)
{
    if (!sv) return bfail(OKPZ_EINVAL, "null server");
    if (quanta) *quanta = sv->quanta;
    if (device_ms) *device_ms = sv->device_ms;
    if (done) *done = sv->done;
    if (bytes_in_use) *bytes_in_use = sv->used;
    return OKPZ_OK;
}

int okpz_serve_free(okpz_server *sv)
{
    if (!sv) return OKPZ_OK;
    if (sv->stream) (void)hipStreamSynchronize(sv->stream);
    for (auto &J : sv->jobs)
        if (J.mem) (void)hipFree(J.mem);
    if (sv->mem) (void)hipFree(sv->mem);
    if (sv->grid_stream) (void)hipStreamSynchronize(sv->grid_stream);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    if (sv->grid_stream) (void)hipStreamDestroy(sv->grid_stream);
    delete sv;
    return OKPZ_OK;
}

}  // extern "C"
