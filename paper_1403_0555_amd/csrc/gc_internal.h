// Internal structures shared by the device kernels and the host runtime of
// the Gribov-copy enumerator.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GC_MAXD 4
#define GC_MAXPT 16        // sites per thread held in registers by the Lanczos step
#define GC_LMAX 512        // Lanczos iteration cap (tridiagonal storage)

// Per-start status codes (mirror GC_START_* of the public header).
#define GC_ST_PENDING 0
#define GC_ST_CONVERGED 1
#define GC_ST_NONCONVERGED 2
#define GC_ST_BADNUM 3
// Internal: converged in single precision, state promoted to double precision
// in HBM, its double-precision phase pending (never left in a finished launch).
#define GC_ST_PROMOTED 0x50

// Copy flags (mirror GC_FLAG_*).
#define GC_F_IN_REGION 1u
#define GC_F_SINGULAR 2u
#define GC_F_SADDLE 4u
#define GC_F_COLLISION 8u
#define GC_F_LANCZOS_CAP 16u
#define GC_F_KEY_OVERFLOW 32u

// Job flags.
#define GC_JOB_SYNC2 4u        // batch-synchronous second pass: start s runs exactly fixed_sweeps[s] sweeps
#define GC_JOB_FROM32 8u       // double-precision pass over the states a single-precision kernel promoted

// Relative spread of F (per site) above which one key is flagged as reached
// by different stationary points.
#define GC_F_SPREAD_PER_SITE 1e-9

// Geometry and link field of one orbit, all in device memory.
struct GcOrbitDev {
    int32_t d, V, K;
    int32_t n_plaq, n_lines, n_elems;
    int32_t ext[GC_MAXD];
    int32_t line_off[GC_MAXD + 1];   // first line index of each direction
    int32_t plane_mu[6], plane_nu[6];
    uint64_t orbit_index;
    const int32_t *coff;             // [K+1] offsets into perm per colour
    const uint16_t *perm;            // [V] sites grouped by colour, ascending inside a colour
    const uint16_t *nbr;             // [2d][V]: forward neighbour of (mu, i) at [mu][i], backward at [d+mu][i]
    const double2 *U64;              // [d][V] (cos phi, sin phi)
    const float2 *U32;               // [d][V] rounded from U64
    const double *phi_plaq;          // [n_plaq] plaquette sums of raw phi
    const double *phi_line;          // [n_lines] line sums of raw phi
    const uint16_t *line_site;       // [n_lines] site of each line with x_mu = 0
};

// Per-start record, 64 bytes, same layout as gc_start_record.
struct GcStartRec {
    int32_t status;
    uint32_t sweeps32, sweeps64, lanczos_iters;
    double F, D, lambda2;
    uint64_t key_hi, key_lo;
    uint32_t paper_X, flags;
};

// Copy-table slot, 64 bytes.  key_hi == 0 marks an empty slot.
struct GcEntry {
    uint64_t key_hi, key_lo;
    uint64_t hits, first_start;
    uint64_t fmin_bits, fmax_bits;   // IEEE bits of F >= 0 order like the values
    uint32_t pad0, pad1;
    uint64_t rep_start;              // lowest start id with F within tolerance of the minimum F
};

// Device counters of one job.
struct GcCounters {
    unsigned long long starts_done, converged, nonconverged, distinct;
    unsigned long long sweeps_total, lanczos_runs, errors, spare;
};

// Compact copy record written by the finalize kernel (same layout as gc_copy).
struct GcCopyRec {
    uint64_t key_hi, key_lo;
    double F, x, lambda2;
    uint64_t hits, first_start, rep_start;
    uint32_t flags, lanczos_iters;
};

// One job (orbit + params + outputs) as seen by the kernels.
struct GcJobDev {
    GcOrbitDev orb;
    double omega, eps32, eps64, lambda_tol;
    int32_t precision, stop_norm, check_every, lanczos_max;
    uint64_t max_sweeps, start_seed, first_start, n_starts;
    uint32_t flags, sync_batch;      // sync_batch: starts per batch of the batch-synchronous stop (0: off)
    GcStartRec *rec;                 // [n_starts]
    GcEntry *table;                  // [table_mask + 1]
    uint64_t table_mask;
    GcCounters *cnt;
    GcCopyRec *copies;               // [n_starts] finalize output
    unsigned long long *n_copies;
    double2 *states;                 // [n_starts][V] final g of every start, natural site order
    uint32_t *blk;                   // [(table_mask + 1) / 256] per-block copy counts, then offsets
    uint32_t *fixed_sweeps;          // [n_starts] batch-synchronous sweep counts (sync_batch > 0), else null
    const double *theta_init;        // [n_starts][V] the caller's start angles, else null (Philox starts)
};

static_assert(sizeof(GcStartRec) == 64, "record layout");
static_assert(sizeof(GcEntry) == 64, "entry layout");
static_assert(sizeof(GcCopyRec) == 72, "copy layout");

// Relax kernel, one workgroup per start (any colouring).
size_t gc_relax_wg_lds_bytes(int V);
hipError_t gc_relax_wg_occupancy(int block, size_t lds_bytes, int *blocks_per_cu);
hipError_t gc_launch_relax_wg(int block, const GcJobDev *jobs, int n_jobs, const uint64_t *prefix,
                              unsigned long long *next, uint64_t total, int grid, size_t lds_bytes, hipStream_t s);

// Post kernels.  Key pass (keys = 1): one workgroup per start, functional,
// key and table insertion.  Filter pass (keys = 0): one workgroup per copy
// of the compacted tables, the FP-operator Lanczos at its representative.
// Workgroup shape for V sites: block threads, sp sites per thread, link
// weights in registers (wreg) or in a global buffer of (d + 3) V doubles per
// workgroup (wbuf, wstride doubles apart).
size_t gc_post_lds_bytes(int d, int V, int keys, int lmax);
void gc_post_shape(int V, int *block, int *sites_per_thread, int *wreg);
hipError_t gc_post_occupancy(int block, int sp, int wreg, int keys, size_t lds_bytes, int *blocks_per_cu);
hipError_t gc_launch_post(int block, int sp, int wreg, int keys, const GcJobDev *jobs, int n_jobs,
                          const uint64_t *prefix, unsigned long long *next, uint64_t total, double *wbuf,
                          uint64_t wstride, int grid, size_t lds_bytes, hipStream_t s);
// Filter pass in the line-segment layout (seg sites per thread along
// direction 0), one kernel per lattice dimension d (every job of a launch
// has dimension d): gc_lanczos_shape returns 0 when no instantiated shape
// fits.  gc_lanczos_form: bit 0 when the segments are whole lines
// (seg == N0), bit 1 when the V/seg threads fit a stride of 7 block / 8
// doubles in the segment-major LDS arrays (else the stride is block); every
// job of a launch has the same form.
int gc_lanczos_shape(int d, const int *ext, int V, int *block, int *seg);
int gc_lanczos_form(int N0, int seg, int V, int block);
// LDS bytes: u and the weight arrays, seg x stride doubles each, then the
// tridiagonal.
size_t gc_lanczos_lds_bytes(int d, int N0, int seg, int V, int lmax, int block);
hipError_t gc_lanczos_occupancy(int d, int block, int seg, int form, size_t lds_bytes, int *blocks_per_cu);
hipError_t gc_launch_lanczos(int d, int block, int seg, int form, const GcJobDev *jobs, int n_jobs,
                             unsigned long long *next, int grid, size_t lds_bytes, hipStream_t s);

// Table and bookkeeping kernels.
hipError_t gc_launch_reset(const GcJobDev *jobs_host, int n_jobs, hipStream_t s);
hipError_t gc_launch_finalize(const GcJobDev *jobs_host, int n_jobs, hipStream_t s);   // representatives + compaction
hipError_t gc_launch_orbit_random(double *phi, int64_t n_links, uint64_t seed, uint64_t orbit_index, hipStream_t s);

// Maximal Abelian reduction of an SU(2) configuration (gc_su2.hip): one
// workgroup; links [d][V] quaternions, nbr [2d][V], csite [V] (colour-0
// sites, then colour-1), phi [d][V] out.  LDS: gc_mag_lds_bytes(V).
struct GcMagOut {
    uint64_t sweeps;
    double R;
    int32_t converged;
    int32_t pad;
};
size_t gc_mag_lds_bytes(int V);
hipError_t gc_launch_mag(const double *links, const int *nbr, const int *csite, int d, int V, double eps,
                         uint64_t max_sweeps, double *phi, GcMagOut *out, hipStream_t s);
hipError_t gc_launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
// Write bytes (host source, copied into kernel arguments) to device memory.
hipError_t gc_launch_store(void *dst, const void *src, size_t bytes, hipStream_t s);
// Per-orbit histogram of the copies of one compacted table: x = F/(dV)
// (quantity 0) or (F - F_g)/F_g against the orbit's lowest F among the
// counted copies (quantity 1); weight 1 per copy or its hit count; only
// copies with all of require_flags; counts [n_bins + 2] (underflow, bins,
// overflow), fmin_bits scratch for F_g.  Enqueued on s.
hipError_t gc_launch_histogram(const GcCopyRec *copies, const unsigned long long *n_copies, double dV, int quantity,
                               int weight_hits, uint32_t require_flags, double lo, double hi, int n_bins,
                               unsigned long long *counts, unsigned long long *fmin_bits, hipStream_t s);
// Batch-synchronous stop: per batch of sync_batch starts, the largest
// first-pass sweep count, written per start to fixed_sweeps; relax counters
// cleared for the second pass.
hipError_t gc_launch_sync(const GcJobDev *jobs_host, int n_jobs, hipStream_t s);

// Value-based count: paper_X < GC_PAPER_VALUES (x <= 2 gives at most 2e8),
// one bit per value.
constexpr uint32_t GC_PAPER_VALUES = 1u << 28;
hipError_t gc_launch_paper_mark(const GcStartRec *rec, uint64_t lo, uint64_t hi, uint32_t *bits,
                                unsigned long long *count, hipStream_t s);
