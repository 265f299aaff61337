/*
 * gribov.h -- C ABI of the MI355X Gribov-copy enumerator for compact U(1).
 *
 * Problem (Mehta & Schroeck, "Enumerating Copies in the First Gribov Region
 * on the Lattice in up to four Dimensions"): on a periodic d-dimensional
 * lattice (Sec. I, compact U(1) paragraph) with link angles phi_{i,mu}, find
 * the local minima over gauge transformations theta of the lattice Landau
 * functional, eq. (3),
 *     F_phi(theta) = sum_{i,mu} (1 - cos(phi_{i,mu} + theta_{i+mu} - theta_i)),
 * by relaxation from many random starts (Sec. III, eqs. (4)-(5)), keep the
 * copies whose Faddeev-Popov operator (the Hessian of eq. (3), Sec. I,
 * lattice Landau gauge paragraph) is positive on the complement of the
 * constant mode (the first Gribov region), and count the distinct ones.
 *
 * Conventions for every entry point:
 *  - Every function returns gc_status: GC_OK (0) or a negative error code.
 *    No C++ exception crosses this boundary.
 *  - Pointers are host pointers unless stated.  Inputs are copied before the
 *    call returns; the caller keeps ownership of every buffer it passes.
 *  - A gc_ctx owns all device memory, streams and kernels it creates.  Calls
 *    on one gc_ctx are serialised internally and may come from any thread.
 *  - A device fault makes the context sticky-failed: later calls return
 *    GC_EDEVICE until gc_destroy; gc_last_error gives the text.
 *  - Site index i = sum_mu x_mu s_mu with s_0 = 1, s_mu = s_{mu-1} N_{mu-1}
 *    (x_0 fastest).  Link (i, mu) has index mu*V + i.
 */
#ifndef GRIBOV_H
#define GRIBOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gc_status;
enum {
    GC_OK = 0,
    GC_EINVAL = -1,        /* bad argument (shape, NaN/Inf angle, null pointer, bad handle) */
    GC_ENOMEM = -2,        /* request larger than the HBM budget, or device memory exhausted */
    GC_EUNSUPPORTED = -3,  /* lattice has no proper colouring (see gc_lattice_check) */
    GC_EDEVICE = -4,       /* HIP runtime or kernel error; context is sticky-failed */
    GC_EBUSY = -5,         /* orbit already has a launch in flight */
    GC_ETIMEOUT = -6,      /* gc_wait timed out; the work continues */
    GC_ENOTFOUND = -7,     /* no such copy */
    GC_ESTATE = -8         /* call not valid in the orbit's current state */
};

/* Precision modes. */
enum { GC_FP64 = 0,        /* every sweep in double precision */
       GC_MIXED = 1 };     /* single-precision sweeps to eps32, then double polish to eps64 */

/* Stopping norms on the lattice divergence div_i = Im(conj(g_i) S_i) (the
 * negative gradient of eq. (3)). */
enum { GC_MEAN_SQ = 0,     /* (1/V) sum_i div_i^2 < eps, per start */
       GC_MAX_ABS = 1 };   /* max_i |div_i| < eps, per start (the paper's rule, Sec. III) */

/* Per-start status. */
enum { GC_START_PENDING = 0, GC_START_CONVERGED = 1, GC_START_NONCONVERGED = 2, GC_START_BADNUM = 3 };

/* Copy flags (first Gribov region test, abstract and Sec. I). */
enum {
    GC_FLAG_IN_REGION = 1,    /* lambda2 > lambda_tol */
    GC_FLAG_SINGULAR = 2,     /* |lambda2| <= lambda_tol */
    GC_FLAG_SADDLE = 4,       /* lambda2 < -lambda_tol */
    GC_FLAG_COLLISION = 8,    /* one key reached with functional values differing by > 1e-9 per site */
    GC_FLAG_LANCZOS_CAP = 16  /* Lanczos stopped at its iteration cap */
};

/* Orbit states reported by gc_poll. */
enum { GC_ORBIT_IDLE = 0, GC_ORBIT_QUEUED = 1, GC_ORBIT_RUNNING = 2, GC_ORBIT_DONE = 3, GC_ORBIT_ERROR = 4 };

typedef struct gc_ctx gc_ctx;   /* opaque */
typedef uint64_t gc_orbit;      /* 0 is never a valid handle */

typedef struct {
    int32_t device;             /* HIP device ordinal */
    int32_t n_streams;          /* streams for concurrent launches (0 -> 4); ignored when hip_stream is set */
    uint64_t hbm_budget_bytes;  /* device bytes the context may hold for orbits, launches and unreleased
                                   results (0 -> 64 GiB); a hard limit */
    void *hip_stream;           /* NULL: the context creates its own streams.  Otherwise a hipStream_t of the
                                   caller (e.g. a PyTorch stream) on params->device: every launch is enqueued
                                   on it, after whatever the caller enqueued before the call, and the caller
                                   keeps ownership (it must outlive the context) */
    const char *tune_cache;     /* NULL or a file path: kernel-variant choices of gc_autotune are read from
                                   it at gc_create and written back after every gc_autotune */
} gc_ctx_params;

typedef struct {
    int32_t dim;                /* 1..4 */
    int32_t extent[4];          /* N_mu >= 2 for mu < dim; V = prod N_mu <= 4096 (a start's state is held on chip) */
    uint32_t antiperiodic;      /* bit mu set: gauge transformations are antiperiodic in direction mu,
                                   g_{i + N_mu e_mu} = -g_i (Sec. II names antiperiodic boundary conditions
                                   beside the periodic ones of Sec. I), which is the periodic problem with
                                   every link that wraps around direction mu multiplied by -1; 0: periodic */
} gc_lattice;

typedef struct {
    double omega;               /* 1: relaxation (eqs. (4)-(5)); (0,2): over-relaxation g <- N((1 - omega) g + omega S/|S|) */
    double eps32;               /* stop of the single-precision phase (GC_MIXED) */
    double eps64;               /* stop of the double-precision phase */
    double lambda_tol;          /* region threshold tau on lambda2 */
    int32_t precision;          /* GC_FP64 or GC_MIXED */
    int32_t stop_norm;          /* GC_MEAN_SQ or GC_MAX_ABS */
    uint32_t check_every;       /* evaluate the stopping norm after every k-th sweep (and at the cap) */
    uint32_t lanczos_max_iter;  /* Lanczos iteration cap (<= 512) */
    uint64_t max_sweeps;        /* per phase; beyond it a start is NONCONVERGED and not keyed */
    uint64_t start_seed;        /* Philox key word for the random starts */
    uint64_t first_start;       /* start ids are first_start .. first_start + n_starts - 1 */
    uint32_t sync_batch;        /* 0: every start stops on its own.  k > 0: the paper's batch-synchronous
                                   stop (Sec. III: the stopping test runs over all concurrently relaxed
                                   samples): the starts of each batch of k consecutive ids all run the same
                                   number of sweeps, the largest of the batch's own stopping sweeps, and a
                                   start is converged if its norm is below eps64 after them.  GC_FP64 only */
    uint32_t pad;
} gc_solve_params;

typedef struct {
    int32_t state;              /* GC_ORBIT_* */
    int32_t pad;
    uint64_t n_starts;          /* of the current or last launch */
    uint64_t starts_done;
    uint64_t converged;
    uint64_t nonconverged;
    uint64_t distinct;          /* distinct keys so far */
    uint64_t in_region;         /* distinct keys with GC_FLAG_IN_REGION (valid when DONE) */
    uint64_t saddles;
    uint64_t singular;
    uint64_t collisions;
    uint64_t sweeps_total;      /* sum over starts of all sweeps (both precisions) */
    uint64_t site_updates;      /* sweeps_total * V */
    uint64_t lanczos_runs;
    uint64_t paper_count;       /* distinct trunc(x * 1e8) over converged starts (valid when DONE) */
    double submit_to_done_ms;   /* latency of the last launch (valid when DONE) */
    double device_ms;           /* device time of the last launch's relax kernel, or of the whole graph of a
                                   batch (valid when DONE) */
    double post_ms;             /* device time of the last launch's key pass and table compaction (single-orbit
                                   launches) */
    double filter_ms;           /* device time of the last launch's FP filter pass (single-orbit launches) */
    uint64_t in_region_hits;    /* converged starts whose copy has GC_FLAG_IN_REGION (valid when DONE) */
    uint64_t lanczos_iters;     /* Lanczos iterations summed over the copies' filter runs (valid when DONE) */
} gc_progress;

/* One distinct copy. */
typedef struct {
    uint64_t key_hi, key_lo;    /* canonical integer key (plaquette and line wrap numbers, hashed) */
    double F;                   /* eq. (3) at the copy's representative: the lowest start id whose F is
                                   within 1e-9 per site of the lowest F reaching the key */
    double x;                   /* F / (d V), in [0, 1] inside the first region */
    double lambda2;             /* lowest eigenvalue of M_FP orthogonal to the constant mode, at the representative */
    uint64_t hits;              /* starts that converged to this key */
    uint64_t first_start;       /* lowest start id reaching it */
    uint64_t rep_start;         /* the representative start (F, lambda2 and gc_fetch_state refer to it) */
    uint32_t flags;             /* GC_FLAG_* */
    uint32_t lanczos_iters;
} gc_copy;

/* One start. */
typedef struct {
    int32_t status;             /* GC_START_* */
    uint32_t sweeps32;
    uint32_t sweeps64;
    uint32_t lanczos_iters;     /* 0 unless this start is the representative of its copy */
    double F;
    double D;                   /* final stopping norm */
    double lambda2;             /* the copy's lambda2 at its representative start, NaN at every other start */
    uint64_t key_hi, key_lo;
    uint32_t paper_X;           /* trunc(x * 1e8) */
    uint32_t flags;             /* GC_FLAG_KEY_OVERFLOW; the lambda2 flags only at a representative */
} gc_start_record;

/* Library version string ("major.minor.patch"). */
const char *gc_version(void);

/* Text for a status code. */
const char *gc_status_str(gc_status s);

/* Validate a lattice (host only, no device needed).  On success stores the
 * number of checkerboard colours K: 2 when every extent is even, else the
 * smallest K >= 3 dividing every extent (Sec. III's two sublattices need
 * even extents).  Returns GC_EINVAL for a bad shape, GC_EUNSUPPORTED when no
 * such K exists.  n_colours may be NULL. */
gc_status gc_lattice_check(const gc_lattice *lat, int32_t *n_colours);

/* Fill *p with the defaults: omega 1, eps32 1e-6, eps64 1e-14, lambda_tol
 * 1e-6, GC_FP64, GC_MEAN_SQ, check_every 1, lanczos_max_iter 300,
 * max_sweeps 100000, start_seed 0, first_start 0. */
gc_status gc_solve_params_default(gc_solve_params *p);

/* Create a context on params->device (NULL params: device 0, defaults). */
gc_status gc_create(const gc_ctx_params *params, gc_ctx **out);

/* Wait for all launches, free every device resource, destroy the context. */
gc_status gc_destroy(gc_ctx *ctx);

/* Load an orbit: phi is [dim][V] link angles in radians (host, float64, any
 * real values; NaN/Inf -> GC_EINVAL).  orbit_index enters the counter of the
 * random starts so that starts of different orbits are independent.  The
 * link field U = exp(i phi) and the orbit's plaquette and line sums of phi
 * (the base of the integer key) are formed once here. */
gc_status gc_orbit_load(gc_ctx *ctx, const gc_lattice *lat, const double *phi,
                        uint64_t orbit_index, gc_orbit *out);

/* Hot orbit at beta = 0 (Sec. I): phi uniform on [-pi, pi), link l = mu V + i
 * drawn by Philox4x64-10 with key (seed, 0), counter (l/4, orbit_index,
 * 0x4F, 0), word l%4, angle = fl(fl(((r>>11) 2^-53) 2pi) - pi). */
gc_status gc_orbit_random(gc_ctx *ctx, const gc_lattice *lat, uint64_t seed,
                          uint64_t orbit_index, gc_orbit *out);

/* SU(2) configurations through the maximal Abelian reduction (Sec. I: eq. (1)
 * states the Landau functional for SU(N_c); the Neuberger problem of SU(N_c)
 * lies in its maximal Abelian subgroup U(1)^{N_c-1}, so its copies are those
 * of a compact U(1) field).  The configuration is gauge-fixed on the coset
 * SU(2)/U(1) to the maximal Abelian gauge, R = sum 1/2 Tr(s3 U' s3 U'^dagger)
 * with U'_{x,mu} = g_x U_{x,mu} g_{x+mu}^dagger maximised site by site
 * (sweeps over colour 0, then colour 1, from g = 1; at each site g_x is the
 * transformation with g_x^dagger s3 g_x along the sum of the rotated s3 of
 * its 2d links, its diagonal element real and non-negative), until the mean
 * over sites of |n_x - n_x^old|^2 in a sweep falls below eps; the phases
 * phi = arg (U')_{11} then load as an ordinary orbit (gc_orbit_load).
 * links: host [dim][V][4] float64 unit quaternions (a0, a1, a2, a3) for
 * U = a0 + i (a1 s1 + a2 s2 + a3 s3); non-finite or |a|^2 off 1 by more than
 * 1e-10, eps < 0 or max_sweeps outside 1 .. 10^6 -> GC_EINVAL.  Even
 * extents, periodic transformations (lat->antiperiodic = 0) and V <= 4096
 * only, else GC_EUNSUPPORTED.  params
 * NULL: eps 1e-20, max_sweeps 100000.  info (may be NULL): sweeps, R/(dim V)
 * and whether the threshold was reached.  Runs on the device, one workgroup,
 * and returns when the orbit is loaded. */
typedef struct gc_mag_params {
    double eps;           /* threshold on the sweep's mean |n - n_old|^2 (>= 0) */
    uint64_t max_sweeps;  /* 1 .. 10^6 */
} gc_mag_params;

typedef struct gc_mag_info {
    uint64_t sweeps;
    double R;             /* R/(dim V), in [-1, 1]; 1 for an Abelian field */
    int32_t converged;
    int32_t reserved;
} gc_mag_info;

gc_status gc_orbit_load_su2(gc_ctx *ctx, const gc_lattice *lat, const double *links,
                            uint64_t orbit_index, const gc_mag_params *params,
                            gc_mag_info *info, gc_orbit *out);

/* Copy the orbit's angles back (host [dim][V]). */
gc_status gc_orbit_angles(gc_ctx *ctx, gc_orbit orbit, double *phi_out);

/* Asynchronously enumerate copies from n_starts random starts (Sec. III):
 * start s draws theta_i by Philox4x64-10 with key (start_seed, 1), counter
 * (i/4, s, orbit_index, 0x53), word i%4, then relaxes it colour by colour
 * until its stopping norm falls below eps, computes F, x, the integer key,
 * inserts the key in the orbit's copy table and, for the lowest start id of
 * each key, the lowest non-constant eigenvalue lambda2 of M_FP by Lanczos.
 * Returns at once: the call only enqueues device work (it never waits for
 * the device).  A launch starts when its bytes fit the context's HBM budget
 * (device memory of running launches and of results not yet released
 * counts) and one of the context's streams is idle; until then it waits in a
 * FIFO queue.  A launch larger than the whole budget is GC_ENOMEM.  A second
 * launch on the same orbit replaces its results (GC_EBUSY while one is in
 * flight).  params NULL: defaults. */
gc_status gc_launch(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const gc_solve_params *params);

/* gc_launch from the caller's gauge transformations instead of random
 * starts: theta [n_starts][V] (host, radians, finite) is start s's angles
 * theta_i, relaxed (at least one sweep) and filtered like a random start.
 * A state that is already stationary stays there after its first sweep, so
 * this also classifies given states: F, key and the first-region flags, e.g.
 * of the trivial orbit's twisted states and singular families (Sec. II).
 * Start ids are first_start .. first_start + n_starts - 1 as usual.  Errors
 * as gc_launch, GC_EINVAL for NULL or non-finite theta. */
gc_status gc_launch_from(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const double *theta,
                         const gc_solve_params *params);

/* Launch several orbits as one batch, captured once into a HIP graph: the
 * orbits are grouped by relax kernel (dimension, layout, slots per lane) and
 * each group is one chain of persistent kernel launches (relax, post,
 * table compaction) in which workgroups claim the group's starts from device
 * counters; the chains are concurrent branches of the graph, so one group's
 * slowest starts overlap the other groups' work.  Relaunching the same
 * orbits with the same start counts and params replays the graph on the
 * same device memory.  Same semantics per orbit as gc_launch; all orbits
 * share params. */
gc_status gc_launch_batch(gc_ctx *ctx, int32_t n_orbits, const gc_orbit *orbits,
                          const uint64_t *n_starts, const gc_solve_params *params);

/* Non-blocking progress of the orbit's current or last launch. */
gc_status gc_poll(gc_ctx *ctx, gc_orbit orbit, gc_progress *out);

/* Block until the orbit's launch is DONE (timeout_ms < 0: forever).
 * GC_ETIMEOUT leaves the launch running.  GC_ENOMEM: the launch is queued
 * and nothing is running, so only gc_release of earlier results can make
 * room for it (it stays queued).  A launch that could not start returns its
 * error (GC_ENOMEM when device memory ran out). */
gc_status gc_wait(gc_ctx *ctx, gc_orbit orbit, int64_t timeout_ms);

/* Distinct copies of a DONE orbit, sorted by (key_hi, key_lo): writes up to
 * cap records from position offset into out, their count to *n_written and
 * the table size to *n_total (either may be NULL). */
gc_status gc_fetch(gc_ctx *ctx, gc_orbit orbit, uint64_t offset, uint64_t cap,
                   gc_copy *out, uint64_t *n_written, uint64_t *n_total);

/* Per-start records of a DONE orbit in start-id order (index 0 is
 * first_start of the launch). */
gc_status gc_fetch_starts(gc_ctx *ctx, gc_orbit orbit, uint64_t offset, uint64_t cap,
                          gc_start_record *out, uint64_t *n_written);

/* Representative gauge transformation of one distinct copy of a DONE orbit
 * (the copy with key (key_hi, key_lo); its representative start is
 * gc_copy.rep_start): writes theta_i - theta_{V-1} wrapped to (-pi, pi] to
 * theta_out [V], the global phase removed by fixing the last site (Sec. I).
 * Errors: GC_EINVAL (bad handle, NULL theta_out), GC_ESTATE (no completed
 * launch), GC_ENOTFOUND (no copy with that key). */
gc_status gc_fetch_state(gc_ctx *ctx, gc_orbit orbit, uint64_t key_hi, uint64_t key_lo, double *theta_out);

/* Final state of any start of the orbit's last (DONE) launch, converged or
 * not, in the same form as gc_fetch_state (theta_i - theta_{V-1}).  Errors:
 * GC_EINVAL (start id outside the launch), GC_ESTATE. */
gc_status gc_fetch_start_state(gc_ctx *ctx, gc_orbit orbit, uint64_t start_id, double *theta_out);

/* Free the orbit and its results (waits for a running launch first; a
 * launch still queued is withdrawn).  Device memory returns to the
 * context's pool, so the call never waits for other launches. */
gc_status gc_release(gc_ctx *ctx, gc_orbit orbit);

/* Sticky error text of the context (always NUL-terminated when cap > 0). */
gc_status gc_last_error(gc_ctx *ctx, char *buf, size_t cap);

/* HBM bytes a gc_launch of n_starts on this orbit would be charged against
 * the context's budget (what admission compares with the free budget). */
gc_status gc_launch_bytes(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const gc_solve_params *params,
                          uint64_t *bytes);

/* The context's HBM budget, the bytes charged by launches that still hold
 * memory, and the number of launches waiting for admission (any may be NULL). */
gc_status gc_memory_info(gc_ctx *ctx, uint64_t *budget, uint64_t *in_use, uint64_t *queued);

/* Device time of the last completed launch's solve kernel in milliseconds,
 * measured with HIP events on the stream the kernel ran on. */
gc_status gc_kernel_time_ms(gc_ctx *ctx, gc_orbit orbit, double *solve_ms);

/* Saturation curve of a completed launch (Sec. III and Figs. 1-3: the
 * number of distinct copies found as the number of random starts grows).
 * For each of the n_points sample sizes N, distinct_out receives the number
 * of copies whose lowest start id lies within the first N starts of the
 * launch (ids first_start .. first_start + N - 1); in_region_only != 0
 * counts only copies flagged GC_FLAG_IN_REGION.  Computed on the host from
 * the fetched copy table.  Caller owns both arrays.  Errors: GC_EINVAL,
 * GC_ESTATE (no completed launch). */
gc_status gc_saturation(gc_ctx *ctx, gc_orbit orbit, int32_t n_points, const uint64_t *sample_sizes,
                        int32_t in_region_only, uint64_t *distinct_out);

/* Histogram quantities and weights of gc_histogram. */
enum { GC_HIST_X = 0,        /* x = F / (d V) of each copy */
       GC_HIST_REL = 1 };    /* (F - F_g) / F_g, F_g the lowest F among the orbit's counted copies */
enum { GC_HIST_COPIES = 0,   /* each distinct copy counts once */
       GC_HIST_STARTS = 1 }; /* each copy counts its hits: the starts that reached it */

/* Distributions of the minima (Sec. IV.B: the normalised distribution of the
 * functional at the minima over orbits and samples, and the distribution of
 * (F_i - F_g)/F_g relative to each orbit's global minimum).  For each of the
 * n_orbits completed launches, the copies carrying every flag of
 * require_flags (e.g. GC_FLAG_IN_REGION) are binned into n_bins equal bins
 * on [lo, hi); counts [n_orbits][n_bins + 2] receives per orbit the
 * underflow count, the bins, then the overflow count (caller-owned).
 * Averages over orbits (e.g. of normalised histograms) are the caller's.
 * Computed on the device from the compacted tables.  Errors: GC_EINVAL,
 * GC_ESTATE (an orbit without a completed launch), GC_ENOMEM. */
gc_status gc_histogram(gc_ctx *ctx, int32_t n_orbits, const gc_orbit *orbits, int32_t quantity, int32_t weight,
                       uint32_t require_flags, double lo, double hi, int32_t n_bins, uint64_t *counts);

/* The paper's own count of a completed launch (Sec. III): the number of
 * distinct values trunc(x * 1e8) among the converged starts within the first
 * N starts of the launch, for each of the n_points sample sizes N (the paper
 * takes N at powers of two; N past n_starts counts every start).  Different
 * copies with equal truncated x count once, and one copy whose starts stopped
 * on either side of a truncation boundary counts twice, so this differs from
 * gc_saturation's count of integer keys.  sample_sizes must be
 * nondecreasing.  Counted on the device, one bit per possible value (a
 * 32 MiB bitmap allocated for the call).  Caller owns both arrays.  Errors:
 * GC_EINVAL (bad arguments, decreasing sizes), GC_ESTATE (no completed
 * launch), GC_ENOMEM. */
gc_status gc_paper_saturation(gc_ctx *ctx, gc_orbit orbit, int32_t n_points, const uint64_t *sample_sizes,
                              uint64_t *distinct_out);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The path
 * of gc_launch for one loaded orbit (same kernels and results), enqueued on
 * hip_stream (NULL: the null stream) without any device or pinned
 * allocation and without waiting for the device.  Working memory is one
 * static device array of 64 MiB per GPU, resident from the library's load
 * until the process ends; every call on a GPU uses the same array and a call
 * clears what it needs, so calls that overlap on one GPU race: keep them on
 * one stream.  It is not charged to the context's HBM budget.
 * Outputs, device memory owned by the caller and written when the stream
 * reaches them: copies_dev[copies_cap] (copies_cap >= n_starts) the
 * distinct copies with the fields of gc_copy, in table order (ascending
 * key_hi except where probing displaced an entry: sort for key order);
 * *n_copies_dev their number; counters_dev NULL or 8 uint64 (starts done,
 * converged, nonconverged, distinct, sweeps total, Lanczos runs, table
 * insert errors, reserved).  The orbit's gc_fetch results are untouched.
 * Errors: GC_EINVAL (bad handle or arguments), GC_ENOMEM (the launch needs
 * more than the static array, e.g. more than about 13000 starts of a 4^4
 * lattice; gc_last_error says how much), launch errors. */
gc_status gc_launch_static(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const gc_solve_params *params,
                           void *hip_stream, gc_copy *copies_dev, uint64_t copies_cap, uint64_t *n_copies_dev,
                           uint64_t *counters_dev);

/* Result of gc_autotune. */
typedef struct {
    int32_t relax_variant;          /* colours whose coefficients a lane keeps in registers (0..2); 0 for
                                       lattices with more than two slots per lane (nothing to tune there) */
    int32_t post_block;             /* FP filter kernel of this lattice: threads per workgroup */
    int32_t post_sites_per_thread;  /* and sites per thread (not tuned: the shape follows from the lattice) */
    int32_t pad;
    double relax_ms, post_ms;       /* best measured times of the chosen variants */
} gc_tune_result;

/* Kernel-variant autotuner for the shape of this orbit (Sec. III sweeps).
 * Runs timed launches of n_starts starts with params on the orbit,
 * synchronously: a warm-up, then, where a lane holds at most two slots per
 * colour, the relax variants that keep the coefficients of 0, 1 or 2 colours
 * in registers, two launches each, timed with HIP events.  The variants
 * compute the same products in the same order, so results are bitwise the
 * same whatever is chosen.  The fastest choice is stored in the context (and
 * in the tuning cache) and used by every later launch of an orbit with the
 * same dimension, slots per lane and precision.  The filter's shape follows
 * from the lattice and is reported, not tuned.  The orbit's results
 * afterwards are those of the last trial launch.  out may be NULL.  Errors:
 * GC_EINVAL (no orbit, n_starts = 0), GC_EBUSY (orbit running), launch
 * errors. */
gc_status gc_autotune(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const gc_solve_params *params,
                      gc_tune_result *out);

#ifdef __cplusplus
}
#endif
#endif /* GRIBOV_H */
