// Post-processing of relaxed starts: one wavefront per start reads the final
// double-precision state g (natural site order) into LDS and forms
//   observables  u_l = conj(g_i) U_l g_{i+mu}, F = sum (1 - Re u_l) (eq. (3)),
//                x = F/(dV) and the paper's X = trunc(x 1e8) (Sec. III);
//   key          plaquette wrap numbers n_p = rint((A_p - Phi_p)/2pi) of the
//                link angles a_l = arg u_l against the orbit's raw plaquette
//                sums, then the line windings, hashed to 128 bits (global
//                phase removed, Sec. I);
//   dedup        open-addressing insert into the orbit's copy table;
//   filter       for the lowest start of a key: Lanczos on the FP operator
//                M = B^T diag(Re u) B (the Hessian of eq. (3)) shifted by
//                sigma 11^T/V, sigma = 4d + 1, whose lowest eigenvalue is the
//                lowest eigenvalue of M off the constant mode (first Gribov
//                region test).
// Also the table bookkeeping kernels: reset, representatives, compaction,
// and the patch of re-filtered representatives.
#include "gc_common.h"

namespace {

using namespace gc;

// Smallest eigenvalue of the k x k tridiagonal (alpha, beta): multisection
// over the 64 lanes on the Sturm count (negative LDL^T pivots).
__device__ double tridiag_min_eig(const double *alpha, const double *beta, int k)
{
    const int lane = threadIdx.x & 63;
    double lo = INFINITY, hi = -INFINITY;
    for (int j = 0; j < k; ++j) {
        const double bl = j > 0 ? fabs(beta[j - 1]) : 0.0;
        const double br = j + 1 < k ? fabs(beta[j]) : 0.0;
        lo = fmin(lo, alpha[j] - bl - br);
        hi = fmax(hi, alpha[j] + bl + br);
    }
    lo -= 1e-12 * (1.0 + fabs(lo));
    hi += 1e-12 * (1.0 + fabs(hi));
    for (int round = 0; round < 24; ++round) {
        const double step = (hi - lo) / 65.0;
        const double x = lo + step * (double)(lane + 1);
        int cnt = 0;
        double q = alpha[0] - x;
        if (q < 0) ++cnt;
        for (int j = 1; j < k; ++j) {
            const double qq = (q == 0.0) ? 1e-300 : q;
            q = (alpha[j] - x) - beta[j - 1] * beta[j - 1] / qq;
            if (q < 0) ++cnt;
        }
        const int first = wave_min_int(cnt >= 1 ? lane : 64);
        const double nlo = (first == 0) ? lo : lo + step * (double)first;
        const double nhi = (first == 64) ? hi : lo + step * (double)(first + 1);
        lo = nlo;
        hi = nhi;
        if (hi - lo <= 1e-15 * fmax(1.0, fabs(hi))) break;
    }
    return 0.5 * (lo + hi);
}

// Insert a key (one lane).  A new key is claimed by CAS on its high word; the
// claimer then publishes the low word.  Returns whether this start is the
// lowest start id seen for the key so far.
__device__ void table_insert(const GcJobDev &J, uint64_t key_hi, uint64_t key_lo, uint64_t sid, double F,
                             bool &claimed, bool &is_min, bool &failed)
{
    claimed = false;
    is_min = false;
    failed = true;
    const uint64_t mask = J.table_mask;
    uint64_t idx = (key_hi ^ (key_hi >> 29)) & mask;
    const uint64_t fbits = (uint64_t)__double_as_longlong(F);
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        GcEntry *e = &J.table[idx];
        const unsigned long long old =
            atomicCAS((unsigned long long *)&e->key_hi, 0ULL, (unsigned long long)key_hi);
        bool match = false;
        if (old == 0ULL) {
            __hip_atomic_store(&e->key_lo, key_lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&e->ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            claimed = true;
            match = true;
        } else if (old == key_hi) {
            // the claimer writes key_lo right after its CAS; bounded wait
            uint32_t rdy = 0;
            for (int spin = 0; spin < (1 << 22); ++spin) {
                rdy = __hip_atomic_load(&e->ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (rdy) break;
                __builtin_amdgcn_s_sleep(2);
            }
            if (!rdy) return;
            match = (__hip_atomic_load(&e->key_lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == key_lo);
        }
        if (match) {
            atomicAdd((unsigned long long *)&e->hits, 1ULL);
            const unsigned long long prev =
                atomicMin((unsigned long long *)&e->first_start, (unsigned long long)sid);
            atomicMin((unsigned long long *)&e->fmin_bits, (unsigned long long)fbits);
            atomicMax((unsigned long long *)&e->fmax_bits, (unsigned long long)fbits);
            is_min = sid < prev;
            failed = false;
            return;
        }
        idx = (idx + 1) & mask;
    }
}

__device__ GcEntry *table_find(const GcJobDev &J, uint64_t key_hi, uint64_t key_lo)
{
    const uint64_t mask = J.table_mask;
    uint64_t idx = (key_hi ^ (key_hi >> 29)) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        GcEntry *e = &J.table[idx];
        if (e->key_hi == 0) return nullptr;
        if (e->key_hi == key_hi && e->key_lo == key_lo) return e;
        idx = (idx + 1) & mask;
    }
    return nullptr;
}

// Lowest eigenvalue of M + sigma 11^T/V by Lanczos without reorthogonalisation
// (extreme Ritz values converge regardless).  q lives in LDS; q_prev and the
// residual in the wave's scratch, each lane touching only its own entries.
__device__ double lanczos_lambda2(const GcJobDev &J, double *vq, const double *sw, double *vp, double *vr,
                                  double *alpha, double *beta, uint32_t &iters, bool &conv)
{
    const int lane = threadIdx.x & 63;
    const GcOrbitDev &O = J.orb;
    const int V = O.V, d = O.d;
    const double sigma = 4.0 * d + 1.0;
    // deterministic start vector orthogonal to the constant mode
    double acc = 0.0;
    for (int i = lane; i < V; i += 64) {
        const double r0 = (double)(mix64((uint64_t)i + 0x5851F42D4C957F2DULL) >> 11) * 0x1.0p-53 - 0.5;
        vr[i] = r0;
        acc += r0;
    }
    const double mean = wave_sum(acc) / (double)V;
    acc = 0.0;
    for (int i = lane; i < V; i += 64) {
        const double r0 = vr[i] - mean;
        vr[i] = r0;
        vp[i] = 0.0;
        acc += r0 * r0;
    }
    const double nrm = sqrt(wave_sum(acc));
    for (int i = lane; i < V; i += 64) vq[i] = vr[i] / nrm;
    wave_sync();
    double beta_prev = 0.0, theta = INFINITY, theta_old = INFINITY;
    const int maxit = min(min(J.lanczos_max, GC_LMAX), V);
    int it = 0;
    conv = false;
    for (it = 0; it < maxit; ++it) {
        double sq = 0.0;
        for (int i = lane; i < V; i += 64) sq += vq[i];
        const double shift = sigma * wave_sum(sq) / (double)V;
        double aq = 0.0;
        for (int i = lane; i < V; i += 64) {
            const double qi = vq[i];
            double m = 0.0;
            for (int mu = 0; mu < d; ++mu) {
                const int f = O.nbr[mu * V + i], b = O.nbr[(d + mu) * V + i];
                m += sw[mu * V + i] * (qi - vq[f]);
                m += sw[mu * V + b] * (qi - vq[b]);
            }
            const double r = m + shift - beta_prev * vp[i];
            vr[i] = r;
            aq += r * qi;
        }
        const double a_j = wave_sum(aq);
        acc = 0.0;
        for (int i = lane; i < V; i += 64) {
            const double r = vr[i] - a_j * vq[i];
            vr[i] = r;
            acc += r * r;
        }
        const double b_j = sqrt(wave_sum(acc));
        if (lane == 0) {
            alpha[it] = a_j;
            beta[it] = b_j;
        }
        wave_sync_global();
        const bool breakdown = b_j <= 1e-13 * sigma;
        if (((it + 1) % 8 == 0) || breakdown || it + 1 == maxit) {
            theta = tridiag_min_eig(alpha, beta, it + 1);
            if (breakdown || fabs(theta - theta_old) <= 1e-12 * fmax(1.0, fabs(theta))) {
                conv = true;
                ++it;
                break;
            }
            theta_old = theta;
        }
        wave_sync();   // every neighbour read of q is done
        for (int i = lane; i < V; i += 64) {
            vp[i] = vq[i];
            vq[i] = vr[i] / b_j;
        }
        beta_prev = b_j;
        wave_sync();
    }
    iters = (uint32_t)it;
    return theta;
}

__device__ uint32_t region_flags(double lam2, double tol)
{
    if (lam2 > tol) return GC_F_IN_REGION;
    if (lam2 < -tol) return GC_F_SADDLE;
    return GC_F_SINGULAR;
}

// One wavefront per workgroup; LDS holds the start's state (16V bytes), later
// reused for the Lanczos vector q.  Scratch per wavefront: alpha, beta, link
// angles [d][V], link weights [d][V], q_prev [V], residual [V].
__global__ __launch_bounds__(64) void post_kernel(const GcJobDev *__restrict__ jobs, int n_jobs,
                                                  const uint64_t *__restrict__ prefix, unsigned long long *next,
                                                  uint64_t total, const unsigned long long *total_dev,
                                                  double *scratch, uint64_t stride)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    if (total_dev) total = *total_dev;
    double *wscr = scratch + (uint64_t)blockIdx.x * stride;
    for (;;) {
        unsigned long long s = 0;
        if (lane == 0) s = atomicAdd(next, 1ULL);
        s = __shfl(s, 0, 64);
        if (s >= total) break;
        int jn = 0;
        if (prefix)
            while (jn + 1 < n_jobs && prefix[jn + 1] <= s) ++jn;
        const GcJobDev &J = jobs[jn];
        const GcOrbitDev &O = J.orb;
        const int V = O.V, d = O.d;
        const bool fixmode = (J.flags & GC_JOB_FIX) != 0;
        const uint64_t local = fixmode ? J.fix[s].start - J.first_start : s - (prefix ? prefix[jn] : 0);
        const uint64_t sid = J.first_start + local;
        GcStartRec rec = J.rec[local];
        if (rec.status != GC_ST_CONVERGED) continue;   // uniform across the wave

        double2 *g = reinterpret_cast<double2 *>(smem);
        const double2 *src = J.states + local * (uint64_t)V;
        for (int i = lane; i < V; i += 64) g[i] = src[i];
        wave_sync();

        double *alpha = wscr;
        double *beta = wscr + GC_LMAX;
        double *sa = wscr + 2 * GC_LMAX;     // [d][V]
        double *sw = sa + (size_t)d * V;     // [d][V]
        double *vp = sw + (size_t)d * V;     // [V]
        double *vr = vp + V;                 // [V]

        // ---- observables
        double facc = 0.0;
        for (int l = lane; l < d * V; l += 64) {
            const int mu = l / V, i = l - mu * V;
            const int f = O.nbr[mu * V + i];
            const double2 u = O.U64[l];
            const double2 gi = g[i], gf = g[f];
            const double tr = u.x * gf.x - u.y * gf.y;
            const double ti = u.x * gf.y + u.y * gf.x;
            const double ur = gi.x * tr + gi.y * ti;
            const double ui = gi.x * ti - gi.y * tr;
            facc += 1.0 - ur;
            sa[l] = atan2(ui, ur);
            sw[l] = ur;
        }
        const double F = wave_sum(facc);
        wave_sync_global();
        uint32_t flags = 0;
        uint64_t key_hi = rec.key_hi, key_lo = rec.key_lo;
        if (!fixmode) {
            // ---- integer key
            const uint64_t c0 = 0x243F6A8885A308D3ULL, c1 = 0x13198A2E03707344ULL;
            uint64_t h0 = 0, h1 = 0;
            int overflow = 0;
            for (int k = lane; k < O.n_elems; k += 64) {
                double val;
                if (k < O.n_plaq) {
                    const int pl = k / V, i = k - pl * V;
                    const int mu = O.plane_mu[pl], nu = O.plane_nu[pl];
                    const int fm = O.nbr[mu * V + i], fn = O.nbr[nu * V + i];
                    const double A = sa[mu * V + i] + sa[nu * V + fm] - sa[mu * V + fn] - sa[nu * V + i];
                    val = rint((A - O.phi_plaq[k]) / kTwoPi);
                } else {
                    const int q = k - O.n_plaq;
                    int mu = 0;
                    while (q >= O.line_off[mu + 1]) ++mu;
                    int i = O.line_site[q];
                    double acc = 0.0;
                    for (int t = 0; t < O.ext[mu]; ++t) {
                        acc += sa[mu * V + i];
                        i = O.nbr[mu * V + i];
                    }
                    val = rint((acc - O.phi_line[q]) / kTwoPi);
                }
                const int e = (int)val;
                if (e < -128 || e > 127) overflow = 1;
                const uint64_t word = ((uint64_t)k << 8) | (uint64_t)(uint8_t)(int8_t)e;
                h0 += mix64(c0 ^ word);
                h1 += mix64(c1 ^ word);
            }
            h0 = wave_sum_u64(h0);
            h1 = wave_sum_u64(h1);
            const int ok = wave_min_int(overflow ? 0 : 1);
            key_hi = mix64(h0 + (uint64_t)O.n_elems);
            key_lo = mix64(h1 + (uint64_t)O.n_elems);
            if (key_hi == 0) key_hi = 1;
            if (!ok) flags |= GC_F_KEY_OVERFLOW;
        }
        // ---- dedup (one lane), then the filter for the lowest start of a key
        int run = fixmode ? 1 : 0;
        if (!fixmode && lane == 0) {
            bool claimed, is_min, failed;
            table_insert(J, key_hi, key_lo, sid, F, claimed, is_min, failed);
            run = is_min ? 1 : 0;
            if (claimed) atomicAdd(&J.cnt->distinct, 1ULL);
            if (failed) atomicAdd(&J.cnt->errors, 1ULL);
        }
        run = __shfl(run, 0, 64);
        double lam2 = NAN;
        uint32_t lit = 0;
        if (run) {
            wave_sync();   // q overwrites the state
            bool conv;
            lam2 = lanczos_lambda2(J, reinterpret_cast<double *>(g), sw, vp, vr, alpha, beta, lit, conv);
            if (!conv) flags |= GC_F_LANCZOS_CAP;
            flags |= region_flags(lam2, J.lambda_tol);
            if (lane == 0) atomicAdd(&J.cnt->lanczos_runs, 1ULL);
        }
        if (lane == 0) {
            if (fixmode) {
                J.fix[s].lambda2 = lam2;
                J.fix[s].flags = flags;
                J.fix[s].lanczos_iters = lit;
            } else {
                rec.F = F;
                rec.key_hi = key_hi;
                rec.key_lo = key_lo;
                rec.paper_X = (uint32_t)(F / ((double)d * (double)V) * 1e8);
                rec.flags = flags;
                rec.lambda2 = lam2;
                rec.lanczos_iters = lit;
                J.rec[local] = rec;
            }
        }
        wave_sync();
    }
}

__global__ void reset_kernel(GcJobDev J)
{
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = gid; t <= J.table_mask; t += stride) {
        GcEntry e;
        e.key_hi = 0;
        e.key_lo = 0;
        e.hits = 0;
        e.first_start = ~0ULL;
        e.fmin_bits = ~0ULL;
        e.fmax_bits = 0;
        e.ready = 0;
        e.pad = 0;
        e.rep_start = ~0ULL;
        J.table[t] = e;
    }
    for (uint64_t t = gid; t < J.n_starts; t += stride) {
        GcStartRec r = {};
        r.lambda2 = NAN;
        J.rec[t] = r;
    }
    if (gid == 0) {
        GcCounters z = {};
        *J.cnt = z;
        *J.n_copies = 0ULL;
        *J.n_fix = 0ULL;
    }
}

// Representative of each copy: the lowest start id whose F is within
// GC_F_SPREAD_PER_SITE per site of the lowest F reaching the key.  A start
// that halted next to a saddle of the same class has a larger F.
__global__ void rep_kernel(GcJobDev J)
{
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const double tolF = GC_F_SPREAD_PER_SITE * (double)J.orb.V;
    for (uint64_t t = gid; t < J.n_starts; t += stride) {
        const GcStartRec r = J.rec[t];
        if (r.status != GC_ST_CONVERGED) continue;
        GcEntry *e = table_find(J, r.key_hi, r.key_lo);
        if (!e) continue;
        const double fmin = __longlong_as_double((long long)e->fmin_bits);
        if (r.F - fmin <= tolF)
            atomicMin((unsigned long long *)&e->rep_start, (unsigned long long)(J.first_start + t));
    }
}

__global__ void compact_kernel(GcJobDev J)
{
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const double dV = (double)J.orb.d * (double)J.orb.V;
    for (uint64_t t = gid; t <= J.table_mask; t += stride) {
        const GcEntry e = J.table[t];
        if (e.key_hi == 0) continue;
        const uint64_t rep = e.rep_start;
        const GcStartRec r = J.rec[rep - J.first_start];
        GcCopyRec c;
        c.key_hi = e.key_hi;
        c.key_lo = e.key_lo;
        c.F = r.F;
        c.x = r.F / dV;
        c.hits = e.hits;
        c.first_start = e.first_start;
        const double fmin = __longlong_as_double((long long)e.fmin_bits);
        const double fmax = __longlong_as_double((long long)e.fmax_bits);
        const uint32_t col = ((fmax - fmin) / (double)J.orb.V > GC_F_SPREAD_PER_SITE) ? GC_F_COLLISION : 0u;
        const unsigned long long slot = atomicAdd(J.n_copies, 1ULL);
        if (rep == e.first_start) {
            // the lowest start ran the filter when it was inserted
            c.lambda2 = r.lambda2;
            c.flags = (r.flags & (GC_F_IN_REGION | GC_F_SINGULAR | GC_F_SADDLE | GC_F_LANCZOS_CAP | GC_F_KEY_OVERFLOW)) | col;
            c.lanczos_iters = r.lanczos_iters;
        } else {
            c.lambda2 = NAN;
            c.flags = col | (r.flags & GC_F_KEY_OVERFLOW);
            c.lanczos_iters = 0;
            const unsigned long long k = atomicAdd(J.n_fix, 1ULL);
            GcFix f;
            f.start = rep;
            f.slot = slot;
            f.lambda2 = NAN;
            f.flags = 0;
            f.lanczos_iters = 0;
            J.fix[k] = f;
        }
        J.copies[slot] = c;
    }
}

__global__ void patch_kernel(GcJobDev J)
{
    const uint64_t n = *J.n_fix;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
        const GcFix f = J.fix[k];
        GcCopyRec &c = J.copies[f.slot];
        c.lambda2 = f.lambda2;
        c.flags |= f.flags & (GC_F_IN_REGION | GC_F_SINGULAR | GC_F_SADDLE | GC_F_LANCZOS_CAP);
        c.lanczos_iters = f.lanczos_iters;
    }
}

__global__ void orbit_random_kernel(double *phi, int64_t n_links, uint64_t seed, uint64_t orbit_index)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * b >= n_links) return;
    uint64_t c[4] = {(uint64_t)b, orbit_index, 0x4FULL, 0ULL};
    philox4x64_10(c, seed, 0ULL);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (4 * b + k < n_links) phi[4 * b + k] = angle_of(c[k]);
}

__global__ void zero_u64_kernel(unsigned long long *p, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0ULL;
}

int grid_for(uint64_t work)
{
    uint64_t g = (work + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

size_t gc_post_lds_bytes(int V) { return 16 * (size_t)V; }

uint64_t gc_post_scratch_doubles(int d, int V) { return 2ull * GC_LMAX + 2ull * d * V + 2ull * V; }

hipError_t gc_post_occupancy(size_t lds_bytes, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, post_kernel, 64, lds_bytes);
}

hipError_t gc_launch_post(const GcJobDev *jobs, int n_jobs, const uint64_t *prefix, unsigned long long *next,
                          uint64_t total, const unsigned long long *total_dev, double *scratch, uint64_t stride,
                          int grid, size_t lds_bytes, hipStream_t s)
{
    hipLaunchKernelGGL(post_kernel, dim3(grid), dim3(64), lds_bytes, s, jobs, n_jobs, prefix, next, total, total_dev,
                       scratch, stride);
    return hipGetLastError();
}

hipError_t gc_launch_reset(const GcJobDev *jobs_host, int n_jobs, hipStream_t s)
{
    for (int j = 0; j < n_jobs; ++j) {
        const GcJobDev &J = jobs_host[j];
        const uint64_t work = J.table_mask + 1 > J.n_starts ? J.table_mask + 1 : J.n_starts;
        hipLaunchKernelGGL(reset_kernel, dim3(grid_for(work)), dim3(256), 0, s, J);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gc_launch_finalize(const GcJobDev *jobs_host, int n_jobs, hipStream_t s)
{
    for (int j = 0; j < n_jobs; ++j) {
        const GcJobDev &J = jobs_host[j];
        hipLaunchKernelGGL(rep_kernel, dim3(grid_for(J.n_starts)), dim3(256), 0, s, J);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(compact_kernel, dim3(grid_for(J.table_mask + 1)), dim3(256), 0, s, J);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gc_launch_patch(const GcJobDev *jobs_host, int n_jobs, hipStream_t s)
{
    for (int j = 0; j < n_jobs; ++j) {
        hipLaunchKernelGGL(patch_kernel, dim3(64), dim3(256), 0, s, jobs_host[j]);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gc_launch_orbit_random(double *phi, int64_t n_links, uint64_t seed, uint64_t orbit_index, hipStream_t s)
{
    const int64_t blocks4 = (n_links + 3) / 4;
    hipLaunchKernelGGL(orbit_random_kernel, dim3((unsigned)((blocks4 + 255) / 256)), dim3(256), 0, s, phi, n_links,
                       seed, orbit_index);
    return hipGetLastError();
}

hipError_t gc_launch_zero_u64(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
