/*
 * okpz -- octahedron-model KPZ growth on AMD MI355X (gfx950).
 *
 * C ABI of the hot path of Kelling & Odor, "Extremely large scale simulation
 * of a KPZ model using graphics cards" (arXiv:1110.6745): Monte Carlo sweeps
 * of the generalized Kawasaki rule (Eq. (1)) on a two-bit-per-site slope
 * lattice (Sec. II) and the exact surface width (Sec. I height
 * reconstruction, Eq. (Wdef)).
 *
 * Conventions shared by every call:
 *  - Return value 0 (OKPZ_OK) on success, a negative OKPZ_E* code otherwise;
 *    okpz_last_error() then gives a message (thread-local).
 *  - A handle is not thread-safe; distinct handles may be used from distinct
 *    threads.  Device work is issued on the handle's HIP stream; calls that
 *    return host results synchronize that stream.
 *  - Lattice sizes: Lx, Ly multiples of 32, 32 <= Lx, Ly <= 2^20.
 *  - Canonical host lattice layout (get/set calls): one byte per site,
 *    row-major, byte[y*Lx + x]; bit 0 = [sigma_x(x,y) = +1], bit 1 =
 *    [sigma_y(x,y) = +1], where sigma_x(x,y) = h(x+1,y) - h(x,y) and
 *    sigma_y(x,y) = h(x,y+1) - h(x,y) on the periodic lattice.
 *  - Heights: h(x,y) = H0 + sum_{k<y} sigma_y(0,k) + sum_{l<x} sigma_x(l,y),
 *    H0 = h(0,0), tracked exactly by the library.
 */
#ifndef OKPZ_H
#define OKPZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OKPZ_OK 0
#define OKPZ_EINVAL (-22)    /* bad argument: size, probability, time, buffer */
#define OKPZ_ENOMEM (-12)    /* device or host allocation failed, buffer too small */
#define OKPZ_EOVERFLOW (-75) /* an exact sum does not fit a signed 64-bit integer */
#define OKPZ_EDEVICE (-5)    /* a HIP runtime error; message kept */
#define OKPZ_EBUSY (-16)     /* resource limit (slots, bytes) reached */

typedef struct okpz_sim okpz_sim; /* opaque; one simulated lattice */

/* Geometry of the two-level dead-border decomposition (Sec. II): block sides
 * Bx, By = largest power of two dividing Lx, Ly, at most 256; thread-cell side
 * C = min(8, Bx, By).  Depends on the lattice size only. */
int okpz_geometry(int64_t Lx, int64_t Ly, int32_t *Bx, int32_t *By, int32_t *C);

/* Device bytes a simulation of this size needs (two lattice copies plus
 * width scratch); what okpz_init_on's buffer must provide. */
size_t okpz_required_bytes(int64_t Lx, int64_t Ly);

/* Create a simulation of an Lx x Ly periodic lattice in the flat zig-zag
 * state h = (x+y) mod 2 (Sec. III: W^2(L,0) = 1/4), time t = 0, attachment
 * probability p and detachment probability q in [0,1] (Eq. (1)), and the
 * seed that keys every random decision.  The library allocates device memory
 * and a stream.  *out receives the handle (NULL on error). */
int okpz_init(okpz_sim **out, int64_t Lx, int64_t Ly, double p, double q, uint64_t seed);

/* As okpz_init, but on caller-owned device memory (dev_buf, at least
 * okpz_required_bytes bytes, 256-byte aligned) and a caller-owned HIP stream
 * (hipStream_t passed as void*, NULL = default stream).  The caller keeps
 * both alive until okpz_free. */
int okpz_init_on(okpz_sim **out, int64_t Lx, int64_t Ly, double p, double q, uint64_t seed,
                 void *dev_buf, size_t bytes, void *hip_stream);

/* Device bytes of a simulation that keeps ONE lattice copy and updates it in
 * place: half the lattice bytes of okpz_required_bytes, which is what lets a
 * 2^20 x 2^20 lattice (2^40 sites, 256 GiB) fit on one 288 GB GPU.  0 for an
 * invalid size. */
size_t okpz_required_bytes_in_place(int64_t Lx, int64_t Ly);

/* As okpz_init_on (dev_buf NULL: the library allocates memory and a stream;
 * otherwise at least okpz_required_bytes_in_place bytes, 256-byte aligned),
 * but with one lattice copy that every sweep updates in place.  The
 * trajectory is the one of a two-copy simulation with the same seed, bit for
 * bit: the blocks of a sweep (Sec. II) cover disjoint sites and each reads
 * and writes only its own, so the order in which blocks run cannot show.
 * Horizontally adjacent blocks share a memory word at their common edge, so
 * a sweep runs as two launches (even and odd block columns; three if the
 * number of block columns is odd).  Every other call works on such a handle
 * as on any other; its checkpoints restore as one-copy simulations. */
int okpz_init_in_place(okpz_sim **out, int64_t Lx, int64_t Ly, double p, double q, uint64_t seed,
                       void *dev_buf, size_t bytes, void *hip_stream);

/* *copies = 2 for a simulation made by okpz_init, okpz_init_on or from a
 * two-copy checkpoint, 1 for one updated in place. */
int okpz_get_copies(const okpz_sim *s, int32_t *copies);

/* Advance by n_mcs >= 0 Monte Carlo steps (Sec. II: one MCS = one overall
 * update, block-decomposition origin moved at every MCS).  Asynchronous on the
 * handle's stream.  Sweep indices must stay below 2^32. */
int okpz_sweep(okpz_sim *s, int64_t n_mcs);

/* Advance to MCS t (t >= current time; t == current time just measures) and
 * return the exact sums sum_h = sum h(x,y) and sum_h2 = sum h(x,y)^2 over all
 * sites (Eq. (Wdef): W^2 = sum_h2/N - (sum_h/N)^2, N = Lx*Ly).  Synchronous.
 * OKPZ_EOVERFLOW if a sum leaves the signed 64-bit range. */
int okpz_width(okpz_sim *s, int64_t t, int64_t *sum_h, int64_t *sum_h2);

/* Same measurement as okpz_width at the current time, returning W^2 in double
 * from the exact integer numerator N*S2 - S1^2 (independent of H0). */
int okpz_w2(okpz_sim *s, double *w2);

/* Power spectrum density of the current surface along the two lattice axes
 * (Sec. III, Eq. (PSD) with h(k) of Eq. (hF), d = 2, normalised by
 * (Lx*Ly)^(-1/2)): sx[n] = |h(k)|^2 at k = (2 pi n/Lx, 0) for n = 0..Lx/2 and
 * sy[n] at k = (0, 2 pi n/Ly) for n = 0..Ly/2; sx[0] = sy[0] = 0 (the mean
 * height is subtracted).  One surface: the ensemble average of Eq. (PSD) and
 * the average over the two directions are the caller's means over calls and
 * over sx, sy.  sx and sy are host arrays of Lx/2+1 and Ly/2+1 doubles; either
 * may be NULL.  The profiles are exact integers; the transform is fp64
 * (radix 2 for a power-of-two side, Bluestein's chirp-z form otherwise).
 * The first call allocates at most min(32 MiB, Lx*Ly/4) + 40*max(Lx,Ly)
 * bytes of device scratch (plus 128*max(Lx,Ly) when a side is not a power of
 * two), kept until okpz_free.  Synchronous. */
int okpz_psd(okpz_sim *s, double *sx, double *sy);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc or hipFree, e.g. a serving loop or a harness that forbids it):
 * okpz_psd without its scratch allocation.  Same arguments and results as
 * okpz_psd, bit for bit; the scratch is a fixed 24 MiB array in device
 * memory, one per GPU, reserved when the library's code is loaded and held
 * until the process ends (its address is looked up once per device when the
 * first handle is created there).  Lattices with a side above 2^17 are
 * rejected with OKPZ_EINVAL.  No call allocates device memory; the result
 * copies to sx and sy go through the HIP runtime's own staging.  Every call
 * on one GPU uses the same array and nothing in it is kept between calls:
 * calls that overlap on one GPU (handles driven from different host threads)
 * race and must be serialised by the caller.  Synchronous. */
int okpz_psd_noalloc(okpz_sim *s, double *sx, double *sy);

/* Current time in MCS, and the absolute height H0 = h(0,0) (synchronous). */
int okpz_time(const okpz_sim *s, int64_t *t);
int okpz_h0(okpz_sim *s, int64_t *h0);

/* The handle's HIP stream (as void*). */
void *okpz_stream(const okpz_sim *s);

/* Copy the whole lattice to host memory in the canonical layout
 * (bytes >= Lx*Ly).  Synchronous. */
int okpz_get_lattice(okpz_sim *s, uint8_t *host, size_t bytes);

/* Copy rows y0 .. y0+nrows-1 (mod Ly) in the canonical layout
 * (bytes >= nrows*Lx).  Synchronous.  For sampled checks of large lattices. */
int okpz_get_rows(okpz_sim *s, int64_t y0, int64_t nrows, uint8_t *host, size_t bytes);

/* Replace the state: canonical lattice (bytes >= Lx*Ly), absolute height H0
 * of site (0,0) and current time t >= 0.  The lattice must be a valid slope
 * field (zero row sums of sigma_x, zero column sums of sigma_y, closed
 * plaquettes), else OKPZ_EINVAL.  Synchronous. */
int okpz_set_lattice(okpz_sim *s, const uint8_t *host, size_t bytes, int64_t H0, int64_t t);

/* Checkpoint: okpz_save writes the full state (parameters, time, H0, packed
 * lattice) to buf; with buf == NULL it only stores the needed size in *bytes.
 * okpz_load creates a new handle from such a buffer; continuing it gives the
 * same trajectory bit for bit as the original. */
int okpz_save(okpz_sim *s, void *buf, size_t *bytes);
int okpz_load(okpz_sim **out, const void *buf, size_t bytes);

/* Execution mapping of the sweep: threads per workgroup (256, 512 or 1024;
 * default 1024), i.e. 4, 2 or 1 thread cells per thread for 256 x 256 blocks.
 * The trajectory does not depend on it: every random decision is keyed by
 * (seed, sweep, block, step, cell), never by thread. */
int okpz_set_threads(okpz_sim *s, int threads);

/* Thread-cell borders of the tiled dynamics (Sec. II).
 * OKPZ_CELLS_DEAD (the default): each 8x8 thread cell draws one of its 7x7
 * sites off its left column and bottom row at every step, so attempts of one
 * step never touch a common bond.
 * OKPZ_CELLS_DELAYED: each cell draws one of all 64 sites; a step first
 * applies the attempts on cell-bulk sites, then those on the cells' left
 * columns and bottom rows, then those on their corners -- the paper's
 * delayed borders, where a thread on its cell's border waits for the bulk
 * updates and corners wait longest.  Block borders stay dead in both.
 * Takes effect from the next sweep; a checkpoint records it.  Both variants
 * are deterministic functions of the seed, each with its own trajectory. */
#define OKPZ_CELLS_DEAD 0
#define OKPZ_CELLS_DELAYED 1
int okpz_set_cell_borders(okpz_sim *s, int32_t kind);
int okpz_get_cell_borders(const okpz_sim *s, int32_t *kind);

/* Wait for the handle's stream. */
int okpz_sync(okpz_sim *s);

/* Release the handle and everything the library allocated for it. */
int okpz_free(okpz_sim *s);

/* Message of the last error on this thread ("" if none). */
const char *okpz_last_error(void);

/* Measurement times of Sec. III: t_{i+1} = (t_i + 10) e^m from t_0 = 0, each
 * rounded up to a whole MCS, repeats dropped, then t_max itself (none for
 * t_max = 0).  These are the times at which batches and servers record
 * widths.  *n receives the number of times; with times != NULL they are
 * written there (cap >= *n entries, else OKPZ_EINVAL).  m in (0, 10],
 * 0 <= t_max < 2^32.  Host only: needs no device. */
int okpz_sampling_times(int64_t t_max, double m, int64_t *times, int64_t cap, int64_t *n);

/* ------------------------------------------------------------------------
 * Batched ensembles: many independent realizations of uneven size, each with
 * its own p, q, seed and length, run to completion in one persistent launch
 * (the paper's ensembles of independent runs, Sec. III and IV).  Each job
 * starts from the flat state and records the exact width sums at the
 * sampling times t_{i+1} = (t_i + 10) e^m (Sec. III; rounded up, duplicates
 * dropped) and at t_max.  A job's trajectory is bit for bit the one the same
 * job gives alone through okpz_init/okpz_sweep.
 * ---------------------------------------------------------------------- */
typedef struct okpz_job {
    int64_t Lx, Ly;   /* multiples of 32 in [32, 8192] */
    double p, q;      /* attachment / detachment probabilities in [0,1] */
    uint64_t seed;
    int64_t t_max;    /* MCS to run, 0 <= t_max < 2^31 */
} okpz_job;

typedef struct okpz_batch okpz_batch; /* opaque */

/* Validate the jobs (OKPZ_EINVAL on a bad job, sampling exponent m outside
 * (0, 10], or more than 65535 jobs) and allocate every job's lattices and
 * sample buffers on the device. */
int okpz_batch_create(okpz_batch **out, const okpz_job *jobs, int32_t n_jobs, double m);

/* Execution mapping of the persistent launch: threads per workgroup (256,
 * 512, 1024) and resident workgroups (0 = two per compute unit).  Results do
 * not depend on it.  Default: 1024 threads when every job has p = 1, q = 0,
 * else 512; two workgroups per compute unit. */
int okpz_batch_set_mapping(okpz_batch *b, int32_t threads, int32_t workgroups);
int okpz_batch_get_mapping(okpz_batch *b, int32_t *threads, int32_t *workgroups);

/* Thread-cell borders of every job of the batch (OKPZ_CELLS_DEAD, the
 * default, or OKPZ_CELLS_DELAYED; see okpz_set_cell_borders).  Applies from
 * the next okpz_batch_run or okpz_batch_autotune; each job's trajectory is the
 * one okpz_sweep gives a lone lattice with the same borders. */
int okpz_batch_set_cell_borders(okpz_batch *b, int32_t kind);
int okpz_batch_get_cell_borders(const okpz_batch *b, int32_t *kind);

/* Pick the mapping by timing every candidate on a scaled-down copy of the
 * workload: the longest job runs trial_mcs sweeps and every other job the
 * same fraction of its own t_max (at least one sweep); results are
 * discarded and the jobs reset.  Keeps the fastest candidate. */
int okpz_batch_autotune(okpz_batch *b, int64_t trial_mcs, int32_t *threads, int32_t *workgroups);

/* Run every job from the flat state to its t_max in one persistent launch.
 * Synchronous.  OKPZ_EDEVICE if the launch's no-progress watchdog fired. */
int okpz_batch_run(okpz_batch *b);

/* The same run in slices, for callers that want control back while a long
 * ensemble runs (progress reports, a deadline of their own): okpz_batch_start
 * resets every job to the flat state; each okpz_batch_run_for then continues
 * the run in one persistent launch whose workgroups stop taking new work
 * once max_ms milliseconds (wall clock, 0 < max_ms <= 3.6e6) have passed,
 * finishing the sweeps they hold, and returns the number of jobs that have
 * reached t_max in *finished.  The run is complete when *finished equals the
 * number of jobs; samples and final states are then those of okpz_batch_run,
 * bit for bit (the slicing only changes when work is done, never which).
 * okpz_batch_last_ms then gives the device time summed over the slices.
 * OKPZ_EINVAL from okpz_batch_run_for without a started run. */
int okpz_batch_start(okpz_batch *b);
int okpz_batch_run_for(okpz_batch *b, double max_ms, int32_t *finished);

/* Device time of the last okpz_batch_run, in milliseconds. */
int okpz_batch_last_ms(okpz_batch *b, float *ms);

/* Samples of one job after a run: count always; with non-NULL arrays of
 * capacity cap, the sampling times t, and exact sum_h, sum_h2 (Eq. (Wdef)). */
int okpz_batch_samples(okpz_batch *b, int32_t job, int64_t *t, int64_t *sum_h, int64_t *sum_h2,
                       int32_t cap, int32_t *count);

/* Histogram of W^2 = sum_h2/N - (sum_h/N)^2 over the samples with t >= t_from
 * of every job of size Lx x Ly: nbins equal bins on [lo, hi) into counts,
 * samples below lo / at or above hi into *under / *over (may be NULL).
 * The steady-state width distribution of Sec. IV comes from such samples. */
int okpz_batch_w2_histogram(okpz_batch *b, int64_t Lx, int64_t Ly, int64_t t_from, double lo,
                            double hi, int32_t nbins, int64_t *counts, int64_t *under, int64_t *over);

/* Steady-state statistics of Sec. IV over the same samples as
 * okpz_batch_w2_histogram (t >= t_from, every job of size Lx x Ly):
 * *count samples; nu[0..3] = non-central moments <(W^2)^n>, n = 1..4;
 * kappa[0..3] = cumulants kappa_1..kappa_4 from them (Eq. (cumulants)).
 * W^2 from the exact integer sums, moments accumulated in extended precision.
 * OKPZ_EINVAL if no sample qualifies. */
int okpz_batch_w2_cumulants(okpz_batch *b, int64_t Lx, int64_t Ly, int64_t t_from, int64_t *count,
                            double *nu, double *kappa);

/* Scaled width distribution Psi_L(x) = <W^2> P_L(W^2 / <W^2>) (Sec. IV) over
 * the same samples: the density of x = W^2 / <W^2> on nbins equal bins of
 * [0, x_hi), psi[i] = (samples in bin i) / (count * bin width); *count =
 * samples used (those with x >= x_hi fall outside every bin). */
int okpz_batch_psi(okpz_batch *b, int64_t Lx, int64_t Ly, int64_t t_from, double x_hi,
                   int32_t nbins, double *psi, int64_t *count);

/* Final state of one job: canonical lattice (bytes >= Lx*Ly) and H0. */
int okpz_batch_get_lattice(okpz_batch *b, int32_t job, uint8_t *host, size_t bytes);
int okpz_batch_h0(okpz_batch *b, int32_t job, int64_t *h0);

int okpz_batch_free(okpz_batch *b);

/* Message of the last batch error on this thread. */
const char *okpz_batch_last_error(void);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of simulation jobs.  Jobs are submitted with
 * an arrival time (seconds on the server's clock; < 0 = now).  Each
 * okpz_serve_step is one quantum: arrived jobs are admitted in arrival order
 * while a slot is free and their device bytes fit hbm_budget (their lattices
 * then stay resident until they finish); one persistent launch advances every
 * resident job by its share of MCS, all jobs' work interleaved on the device;
 * finished jobs are retired and their memory freed.  A quantum lasts about
 * quantum_sites / 1e12 seconds; a job's share is the number of its sweeps
 * (at least one) that fit that time, a sweep of an L x L lattice counted as
 * 20 us + L^2 / 1e12 s.  Results are bit for bit those of the job run alone. 
 * ---------------------------------------------------------------------- */
typedef struct okpz_server okpz_server; /* opaque */

int okpz_serve_create(okpz_server **out, size_t hbm_budget, int32_t max_slots,
                      int64_t quantum_sites, double m);
int okpz_serve_set_mapping(okpz_server *sv, int32_t threads, int32_t workgroups);
/* Thread-cell borders (OKPZ_CELLS_DEAD, the default, or OKPZ_CELLS_DELAYED,
 * Sec. II) of every job of the server; set before the first okpz_serve_submit
 * (OKPZ_EINVAL afterwards).  Each job's result is then that of a lone
 * simulation with the same borders. */
int okpz_serve_set_cell_borders(okpz_server *sv, int32_t kind);
int okpz_serve_get_cell_borders(const okpz_server *sv, int32_t *kind);
/* Seconds since the server was created. */
int okpz_serve_now(okpz_server *sv, double *now);
/* Queue a job; OKPZ_EBUSY if it could never fit the budget.  keep_lattice:
 * keep the final lattice on the host for okpz_serve_result. */
int okpz_serve_submit(okpz_server *sv, const okpz_job *job, double arrival_s, int32_t keep_lattice,
                      int64_t *id);
/* One quantum (admission, one launch, retirement).  Returns at once with
 * *running = 0 if nothing is resident. */
int okpz_serve_step(okpz_server *sv, int32_t *running, int32_t *waiting);
/* Job status (0 waiting, 1 running, 2 done, 3 cancelled) and its clock
 * times (-1 if not yet; a cancelled job's finish time is when it was
 * cancelled). */
int okpz_serve_job(okpz_server *sv, int64_t id, int32_t *state, double *arrival, double *admit,
                   double *finish);
/* Withdraw a job: a waiting job is never admitted; a running one is retired
 * at once (between quanta), keeping the samples recorded so far, its H0 and,
 * if it asked to keep it, its lattice at the MCS it had reached, and its
 * device memory and slot are freed for other jobs.  Its state becomes 3.
 * OKPZ_EINVAL for an unknown job or one that has finished or was cancelled. */
int okpz_serve_cancel(okpz_server *sv, int64_t id);
/* Samples of a finished job (as okpz_batch_samples); of a cancelled job,
 * those recorded before the cancellation (count 0 if it never ran). */
int okpz_serve_samples(okpz_server *sv, int64_t id, int64_t *t, int64_t *sum_h, int64_t *sum_h2,
                       int32_t cap, int32_t *count);
/* Final H0 and, if kept, the canonical final lattice of a finished job (of a
 * job cancelled while running: at the MCS it had reached). */
int okpz_serve_result(okpz_server *sv, int64_t id, uint8_t *host, size_t bytes, int64_t *h0);
/* Quanta run, device milliseconds, jobs done (cancelled ones not counted), device bytes held
 * by jobs. */
int okpz_serve_stats(okpz_server *sv, int64_t *quanta, double *device_ms, int64_t *done,
                     size_t *bytes_in_use);
int okpz_serve_free(okpz_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* OKPZ_H */
