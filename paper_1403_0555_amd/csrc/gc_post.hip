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
#include "gc_filter.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {

using namespace gc;

// Home slot of a key: the top bits of key_hi (uniformly distributed), so
// that table order is key order up to the displacement of linear probing.
__device__ __forceinline__ uint64_t table_home(uint64_t key_hi, uint64_t mask)
{
    const int b = __popcll(mask);
    return b ? (key_hi >> (64 - b)) : 0;
}

// Insert a key (one lane).  A new key is claimed by CAS on its high word; the
// claimer then writes the low word, which is never zero, so zero means "not
// written yet" to a start that finds the high word.  Only relaxed atomics are
// used: an agent-scope acquire or release would write back or invalidate the
// whole L2 of the XCD.  Nothing else is published through the entry before
// the kernel ends (hits, ids and F bounds are atomics read by later kernels).
// Returns whether this start is the lowest start id seen for the key so far.
__device__ void table_insert(const GcJobDev &J, uint64_t key_hi, uint64_t key_lo, uint64_t sid, double F,
                             bool &claimed, bool &is_min, bool &failed)
{
    claimed = false;
    is_min = false;
    failed = true;
    const uint64_t mask = J.table_mask;
    uint64_t idx = table_home(key_hi, mask);
    const uint64_t fbits = (uint64_t)__double_as_longlong(F);
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        GcEntry *e = &J.table[idx];
        const unsigned long long old =
            atomicCAS((unsigned long long *)&e->key_hi, 0ULL, (unsigned long long)key_hi);
        bool match = false;
        if (old == 0ULL) {
            __hip_atomic_store(&e->key_lo, key_lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            claimed = true;
            match = true;
        } else if (old == key_hi) {
            // the claimer writes key_lo right after its CAS; bounded wait
            uint64_t lo = 0;
            for (int spin = 0; spin < (1 << 22); ++spin) {
                lo = __hip_atomic_load(&e->key_lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (lo != 0) break;
                __builtin_amdgcn_s_sleep(2);
            }
            if (lo == 0) return;
            match = (lo == key_lo);
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
    uint64_t idx = table_home(key_hi, mask);
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        GcEntry *e = &J.table[idx];
        if (e->key_hi == 0) return nullptr;
        if (e->key_hi == key_hi && e->key_lo == key_lo) return e;
        idx = (idx + 1) & mask;
    }
    return nullptr;
}

// Values at a thread's own sites i = tid + B k: registers, or a strided
// view of the workgroup's global slice.
template <bool REG, int SP> struct OwnVec;
template <int SP> struct OwnVec<true, SP> {
    double v[SP];
    __device__ __forceinline__ double get(int k) const { return v[k]; }
    __device__ __forceinline__ void set(int k, double x) { v[k] = x; }
};
template <int SP> struct OwnVec<false, SP> {
    glb_ptr<double> p;
    int stride;
    __device__ __forceinline__ double get(int k) const { return p[k * stride]; }
    __device__ __forceinline__ void set(int k, double x) { p[k * stride] = x; }
};

// Post pass over the relaxed starts (KEYS) or filter pass over the copies of
// the compacted tables (!KEYS), one workgroup of B threads per item; thread t
// owns sites i = t + B k, k < SP.
//   KEYS: observables (F, x, the paper's X), the integer key and the table
//         insert of every converged start.
//   !KEYS: for each distinct copy, the FP filter at its representative
//         start: Lanczos on A = M + sigma 11^T/V.  With WREG the link weights,
//         neighbour indices and the entries of q_prev and M u of the own sites
//         stay in registers; otherwise they live in the workgroup's slice of
//         wbuf ((d + 3) V doubles: forward link weights, then q_prev and M u).
//         This is the general layout; lanczos_kernel below is the faster one
//         for the shapes it is instantiated for.
// LDS: the state g (16V bytes, later the Lanczos vector u), then the link
// angles as floats (4dV bytes) during the key, or the tridiagonal.
// The angle of a link is atan2 in single precision: the branch cut at +-pi is
// decided by the sign of Im u alone, which rounding keeps, and a plaquette or
// line sum then lies within about 1e-5 of its multiple of 2pi, so the wrap
// numbers are the ones double precision gives.
template <int B, int SP, bool WREG, bool KEYS>
__global__ __launch_bounds__(B) void post_kernel(const GcJobDev *__restrict__ jobs, int n_jobs,
                                                 const uint64_t *__restrict__ prefix, unsigned long long *next,
                                                 uint64_t total, double *wbuf_all, uint64_t wstride)
{
    constexpr int NW = (WREG && !KEYS) ? SP : 1;   // register weights per thread (dummy otherwise)
    constexpr int NN = (WREG && !KEYS) ? SP : 1;   // register neighbour words per thread
    glb_ptr<double> wbuf = as_global(wbuf_all + (WREG ? 0 : (uint64_t)blockIdx.x * wstride));
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[2 * 4 * (B / 64)];
    __shared__ uint64_t ured[2 * (B / 64)];
    __shared__ int ired[2 * (B / 64)];
    int rph = 0, uph = 0, iph = 0;   // halves of the reduction scratch in use
    __shared__ unsigned long long claim;
    for (;;) {
        // re-derived per item so that nothing indexed by it is hoisted out of
        // the item loop and held in registers across it
        const int tid = (int)threadIdx.x + opaque_zero();
        if (tid == 0) claim = atomicAdd(next, 1ULL);
        __syncthreads();
        const uint64_t s = uniform((uint64_t)claim);
        __syncthreads();
        int jn = 0;
        uint64_t local = 0, c = 0;
        if constexpr (KEYS) {
            if (s >= total) break;
            while (jn + 1 < n_jobs && prefix[jn + 1] <= s) ++jn;
            jn = uniform(jn);
            local = s - prefix[jn];
        } else {
            // copies of the jobs' tables, in job order
            uint64_t base = 0;
            jn = -1;
            for (int j = 0; j < n_jobs; ++j) {
                const uint64_t nc = *jobs[j].n_copies;
                if (s < base + nc) {
                    jn = j;
                    break;
                }
                base += nc;
            }
            jn = uniform(jn);
            if (jn < 0) break;
            c = s - base;
            local = jobs[jn].copies[c].rep_start - jobs[jn].first_start;
        }
        const GcJobDev &J = jobs[jn];
        const GcOrbitDev &O = J.orb;
        const int V = O.V, d = O.d;
        const uint64_t sid = J.first_start + local;
        const GcStartRec rec0 = J.rec[local];
        if (KEYS && rec0.status != GC_ST_CONVERGED) continue;   // uniform across the workgroup

        // the filter stages the state in LDS, followed by the tridiagonal;
        // the key pass reads it from global memory (once per link end, the
        // start's few kilobytes staying in cache) and keeps only the link
        // angles in LDS, so that more workgroups share a CU
        lds_ptr<dbl2> g = as_lds(reinterpret_cast<dbl2 *>(smem));
        lds_ptr<float> a32 = as_lds(reinterpret_cast<float *>(smem));
        lds_ptr<double> alpha = as_lds(reinterpret_cast<double *>(smem + 16 * (size_t)V));
        const int lmax = min(min(J.lanczos_max, GC_LMAX), V);
        lds_ptr<double> beta2 = alpha + lmax;
        glb_ptr<const dbl2> src = as_global(reinterpret_cast<const dbl2 *>(J.states + local * (uint64_t)V));
        if constexpr (!KEYS) {
            for (int i = tid; i < V; i += B) g[i] = src[i];
            __syncthreads();
        }

        // ---- own sites: forward links (F, angles) for the key, or the FP
        // weights w = Re u of every link touching the site for the filter
        glb_ptr<const dbl2> U = as_global(reinterpret_cast<const dbl2 *>(O.U64));
        double wf[NW][GC_MAXD], wb[NW][GC_MAXD];
        uint32_t nfb[NN][GC_MAXD];   // forward | backward << 16
        double facc = 0.0;
#pragma unroll
        for (int k = 0; k < SP; ++k) {
            const int i = tid + B * k;
#pragma unroll
            for (int mu = 0; mu < GC_MAXD; ++mu) {
                if (WREG && !KEYS) {
                    wf[k % NW][mu] = 0.0;
                    wb[k % NW][mu] = 0.0;
                    nfb[k % NN][mu] = 0;
                }
                if (i < V && mu < d) {
                    const int f = O.nbr[mu * V + i], b = O.nbr[(d + mu) * V + i];
                    const dbl2 gi = KEYS ? src[i] : g[i], gf = KEYS ? src[f] : g[f];
                    const dbl2 u = U[mu * V + i];
                    const double tr = u.x * gf.x - u.y * gf.y, ti = u.x * gf.y + u.y * gf.x;
                    const double ur = gi.x * tr + gi.y * ti, ui = gi.x * ti - gi.y * tr;
                    if constexpr (KEYS) {
                        facc += 1.0 - ur;
                        a32[mu * V + i] = atan2f((float)ui, (float)ur);
                    } else {
                        if (WREG) {
                            nfb[k % NN][mu] = (uint32_t)f | ((uint32_t)b << 16);
                            wf[k % NW][mu] = ur;
                            const dbl2 gb = g[b];
                            const dbl2 v = U[mu * V + b];
                            const double sr = v.x * gi.x - v.y * gi.y, si = v.x * gi.y + v.y * gi.x;
                            wb[k % NW][mu] = gb.x * sr + gb.y * si;
                        } else {
                            wbuf[mu * V + i] = ur;
                        }
                    }
                }
            }
        }
        if constexpr (KEYS) {
            double tmp1[1] = {facc};
            wg_sum_n<B, 1>(tmp1, red, rph);
            const double F = tmp1[0];
            __syncthreads();   // angles visible to the whole workgroup
            uint32_t flags = 0;
            // ---- integer key: plaquette wrap numbers, then line windings
            const uint64_t c0 = 0x243F6A8885A308D3ULL, c1 = 0x13198A2E03707344ULL;
            uint64_t h0 = 0, h1 = 0;
            int overflow = 0;
            // one element: its wrap number e into both hash lanes
            auto fold = [&](int k, double val) {
                const int e = (int)val;
                if (e < -128 || e > 127) overflow = 1;
                const uint64_t word = ((uint64_t)k << 8) | (uint64_t)(uint8_t)(int8_t)e;
                h0 += mix64(c0 ^ word);
                h1 += mix64(c1 ^ word);
            };
            // plaquettes: planes in order (uniform), sites across the threads
            // (the wrap numbers lie within about 1e-5 of integers, so the
            // quotient by 2 pi may be a product with its reciprocal; the
            // hash sums commute, so the order of the elements is free)
            constexpr double kInvTwoPi = 1.0 / kTwoPi;
            for (int pl = 0; pl < O.n_plaq / V; ++pl) {
                const int mu = O.plane_mu[pl], nu = O.plane_nu[pl];
#pragma unroll 2
                for (int i = tid; i < V; i += B) {
                    const int fm = O.nbr[mu * V + i], fn = O.nbr[nu * V + i];
                    const double A = (double)a32[mu * V + i] + (double)a32[nu * V + fm] - (double)a32[mu * V + fn] -
                                     (double)a32[nu * V + i];
                    const int k = pl * V + i;
                    fold(k, rint((A - O.phi_plaq[k]) * kInvTwoPi));
                }
            }
            // line windings: lines of direction mu in order; a line starts
            // at its site with x_mu = 0 and steps by the site stride of mu
            int st = 1;
            for (int mu = 0; mu < d; ++mu) {
                for (int q = O.line_off[mu] + tid; q < O.line_off[mu + 1]; q += B) {
                    int i = O.line_site[q];
                    double acc = 0.0;
                    for (int t = 0; t < O.ext[mu]; ++t) {
                        acc += (double)a32[mu * V + i];
                        i += st;
                    }
                    fold(O.n_plaq + q, rint((acc - O.phi_line[q]) * kInvTwoPi));
                }
                st *= O.ext[mu];
            }
            h0 = wg_sum_u64<B>(h0, ured, uph);
            h1 = wg_sum_u64<B>(h1, ured, uph);
            const int ok = wg_min_int<B>(overflow ? 0 : 1, ired, iph);
            uint64_t key_hi = mix64(h0 + (uint64_t)O.n_elems);
            uint64_t key_lo = mix64(h1 + (uint64_t)O.n_elems);
            if (key_hi == 0) key_hi = 1;
            if (key_lo == 0) key_lo = 1;
            if (!ok) flags |= GC_F_KEY_OVERFLOW;
            if (tid == 0) {
                bool claimed, is_min, failed;
                table_insert(J, key_hi, key_lo, sid, F, claimed, is_min, failed);
                if (claimed) atomicAdd(&J.cnt->distinct, 1ULL);
                if (failed) atomicAdd(&J.cnt->errors, 1ULL);
                GcStartRec rc = rec0;
                rc.F = F;
                rc.key_hi = key_hi;
                rc.key_lo = key_lo;
                rc.paper_X = (uint32_t)(F / ((double)d * (double)V) * 1e8);
                rc.flags = flags;
                rc.lambda2 = NAN;
                rc.lanczos_iters = 0;
                J.rec[local] = rc;
            }
            __syncthreads();
            continue;
        }
        uint32_t flags = 0;
        double lam2 = NAN;
        uint32_t lit = 0;
        {
            // ---- Lanczos on A = M + sigma 11^T/V, M = B^T diag(w) B, with one
            // reduction per iteration.  The vector u in LDS (over the state) is
            // the unnormalised residual r_{j-1} of the previous iteration (the
            // mean-free start vector at first); its norm beta_{j-1} comes out of
            // this iteration's reduction together with u.(M u), sum u and
            // u.q_{j-2}, and then q_j = u/beta, M q_j = (M u)/beta,
            // alpha_j = q_j.(A q_j) - beta_{j-1} q_j.q_{j-1} and the residual
            // r_j = A q_j - beta_{j-1} q_{j-1} - alpha_j q_j follow site by site.
            // q_{j-1} and M u of the own sites stay in registers.
            const double sigma = 4.0 * d + 1.0;
            const double sigma_v = sigma / (double)V;   // the weight of the projector on the constant vector
            lds_ptr<double> vu = as_lds(reinterpret_cast<double *>(smem));
            OwnVec<WREG, SP> qp, mu;
            if constexpr (!WREG) {
                qp.p = wbuf + (size_t)d * V + tid;
                mu.p = qp.p + V;
                qp.stride = mu.stride = B;
            }
            double sums[1] = {0.0};
#pragma unroll
            for (int k = 0; k < SP; ++k) {
                const int i = tid + B * k;
                if (i < V) {
                    const double x = (double)(mix64((uint64_t)i + 0x5851F42D4C957F2DULL) >> 11) * 0x1.0p-53 - 0.5;
                    qp.set(k, 0.0);
                    mu.set(k, x);
                    sums[0] += x;
                }
            }
            wg_sum_n<B, 1>(sums, red, rph);
            const double mean = sums[0] / (double)V;
            if (B > 64) __syncthreads();   // every thread is done with g before u overwrites it
            else wave_sync();
#pragma unroll
            for (int k = 0; k < SP; ++k) {
                const int i = tid + B * k;
                if (i < V) vu[i] = mu.get(k) - mean;
            }
            double theta = INFINITY, theta_old = INFINITY, theta_step = 1.0;
            double rows_lo = INFINITY, rows_hi = -INFINITY;   // Gershgorin bounds of the complete rows
            double a_prev = 0.0, b_prev2 = 0.0;                // alpha_{j-1}, beta_{j-2}
            int next_check = kFirstCheck;                      // iteration count of the next Ritz check
            int it = 0;
            bool conv = false;
            for (it = 0; it < lmax; ++it) {
                if (B > 64) __syncthreads();   // u complete in LDS
                else wave_sync();
                // per-iteration copy of the thread index: the site addresses are
                // recomputed each iteration instead of being held in registers
                const int ti = tid + opaque_zero();
                // (M u)_i for the own sites, then u.u, u.Mu, sum u, u.q_prev at once
                double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 0; k < SP; ++k) {
                    const int i = ti + B * k;
                    if (i < V) {
                        const double ui = vu[i];
                        double m = 0.0;
#pragma unroll
                        for (int mu_ = 0; mu_ < GC_MAXD; ++mu_)
                            if (mu_ < d) {
                                uint32_t f, b;
                                double w1, w2;
                                if constexpr (WREG) {
                                    f = nfb[k % NN][mu_] & 0xFFFFu;
                                    b = nfb[k % NN][mu_] >> 16;
                                    w1 = wf[k % NW][mu_];
                                    w2 = wb[k % NW][mu_];
                                } else {
                                    f = O.nbr[mu_ * V + i];
                                    b = O.nbr[(d + mu_) * V + i];
                                    w1 = wbuf[mu_ * V + i];
                                    w2 = wbuf[mu_ * V + b];
                                }
                                m += w1 * (ui - vu[f]) + w2 * (ui - vu[b]);
                            }
                        mu.set(k, m);
                        s4[0] += ui * ui;
                        s4[1] += ui * m;
                        s4[2] += ui;
                        s4[3] += ui * qp.get(k);
                    }
                    // one site at a time: keeps the scheduler from holding
                    // every neighbour of every own site in registers
                    __builtin_amdgcn_sched_barrier(0);
                }
                wg_sum_n<B, 4>(s4, red, rph);
                // 1/|u| through the reciprocal square root (a vanishing |u|
                // gives bt = 0), as in the line-segment kernel
                const double inv = rsq(fmax(s4[0], 1e-300));
                const double bt = s4[0] * inv;
                const double bp = it > 0 ? bt : 0.0;      // beta_{j-1} (the start vector's norm is not in T)
                if (it > 0) {
                    if (tid == 0) beta2[it - 1] = s4[0];
                    // row it - 1 of T now has both neighbours
                    rows_lo = fmin(rows_lo, a_prev - b_prev2 - bt);
                    rows_hi = fmax(rows_hi, a_prev + b_prev2 + bt);
                    if (bt <= 1e-13 * sigma) {
                        // the Krylov space is exhausted: T of it rows is exact
                        if (B > 64) __syncthreads();
                        else wave_sync();
                        double theta_hi;
                        theta = ritz_min<B>(alpha, beta2, it, rows_lo, rows_hi, theta_old, theta_step, ired, iph,
                                            kRitzTol, true, theta_hi);
                        conv = true;
                        break;
                    }
                }
                const double sq = s4[2] * inv;
                const double shift = sigma_v * sq;
                const double a_j = s4[1] * inv * inv + shift * sq - bp * (s4[3] * inv);
                if (tid == 0) alpha[it] = a_j;
                // the residual over u: every thread finished reading u in the
                // reduction above
#pragma unroll
                for (int k = 0; k < SP; ++k) {
                    const int i = ti + B * k;
                    if (i < V) {
                        const double q = vu[i] * inv;
                        const double r = mu.get(k) * inv + shift - bp * qp.get(k) - a_j * q;
                        qp.set(k, q);
                        vu[i] = r;
                    }
                }
                if (it + 1 >= next_check || it + 1 == lmax) {
                    if (B > 64) __syncthreads();   // the tridiagonal is complete in LDS
                    else wave_sync();
                    const bool final = it + 1 == lmax;
                    double theta_hi;
                    theta = ritz_min<B>(alpha, beta2, it + 1, fmin(rows_lo, a_j - bp), fmax(rows_hi, a_j + bp),
                                        theta_old, theta_step, ired, iph, kRitzTol, final, theta_hi);
                    const double tol = kRitzTol * fmax(1.0, fabs(theta));
                    // theta_old is an upper bound of the previous value, so this
                    // change is at least the true one
                    const double change = theta_old - theta;
                    if (fabs(change) <= tol) {
                        conv = true;
                        ++it;
                        break;
                    }
                    // far from converged: look again later (the change is then
                    // measured over the longer gap, a test at least as strict)
                    const int gap = check_gap(change, tol);
                    next_check = it + 1 + gap;
                    if (theta_old < INFINITY) theta_step = change;
                    theta_old = theta_hi;
                }
                b_prev2 = bp;
                a_prev = a_j;
            }
            lam2 = theta;
            lit = (uint32_t)it;
            if (!conv) flags |= GC_F_LANCZOS_CAP;
            flags |= region_flags(lam2, J.lambda_tol);
            if (tid == 0) atomicAdd(&J.cnt->lanczos_runs, 1ULL);
                }
        if (tid == 0) write_filter(J, c, local, lam2, flags, lit);
        __syncthreads();
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
        e.pad0 = 0;
        e.pad1 = 0;
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

// Ordered compaction of the table into the copy list, in three passes
// over blocks of 256 slots: count the occupied slots of each block, scan the
// counts, scatter each block's copies in slot order.

__global__ __launch_bounds__(256) void count_kernel(GcJobDev J)
{
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const int occ = (t <= J.table_mask && J.table[t].key_hi != 0) ? 1 : 0;
    const int n = __syncthreads_count(occ);
    if (threadIdx.x == 0) J.blk[blockIdx.x] = (uint32_t)n;
}

// One workgroup: exclusive scan of the block counts in chunks of 1024, the
// total into n_copies.
__global__ __launch_bounds__(1024) void scan_kernel(GcJobDev J, uint32_t nblk)
{
    __shared__ uint32_t buf[1024];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nblk; base += 1024) {
        const uint32_t k = base + threadIdx.x;
        const uint32_t v = k < nblk ? J.blk[k] : 0u;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t add = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0u;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (k < nblk) J.blk[k] = carry + buf[threadIdx.x] - v;
        carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *J.n_copies = carry;
}

__global__ __launch_bounds__(256) void scatter_kernel(GcJobDev J)
{
    __shared__ uint32_t wave_off[4];
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const bool occ = t <= J.table_mask && J.table[t].key_hi != 0;
    const uint64_t ball = __ballot(occ);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t below = (uint32_t)__popcll(ball & ((1ull << lane) - 1ull));
    if (lane == 0) wave_off[wave] = (uint32_t)__popcll(ball);
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += wave_off[w];
    if (!occ) return;
    const uint64_t slot = (uint64_t)J.blk[blockIdx.x] + pre + below;
    const double dV = (double)J.orb.d * (double)J.orb.V;
    const GcEntry e = J.table[t];
    const uint64_t rep = e.rep_start;
    const GcStartRec r = J.rec[rep - J.first_start];
    GcCopyRec c;
    c.key_hi = e.key_hi;
    c.key_lo = e.key_lo;
    c.F = r.F;
    c.x = r.F / dV;
    c.hits = e.hits;
    c.first_start = e.first_start;
    c.rep_start = rep;
    const double fmin = __longlong_as_double((long long)e.fmin_bits);
    const double fmax = __longlong_as_double((long long)e.fmax_bits);
    const uint32_t col = ((fmax - fmin) / (double)J.orb.V > GC_F_SPREAD_PER_SITE) ? GC_F_COLLISION : 0u;
    // the filter pass fills in lambda2, its flags and iterations
    c.lambda2 = NAN;
    c.flags = col | (r.flags & GC_F_KEY_OVERFLOW);
    c.lanczos_iters = 0;
    J.copies[slot] = c;
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

// Batch-synchronous stop (Sec. III: one stopping test over all samples
// relaxed together): after a first pass in which every start stopped on its
// own, each start of the batch [b k, (b + 1) k) of the launch gets the
// batch's largest sweep count; the second pass runs exactly that many.  The
// relax counters are cleared so that they count the second pass.
__global__ void sync_kernel(GcJobDev J)
{
    const uint64_t k = J.sync_batch;
    const uint64_t nb = (J.n_starts + k - 1) / k;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += stride) {
        const uint64_t lo = b * k, hi = min(J.n_starts, lo + k);
        uint32_t T = 0;
        for (uint64_t s = lo; s < hi; ++s) T = max(T, J.rec[s].sweeps64);
        for (uint64_t s = lo; s < hi; ++s) J.fixed_sweeps[s] = T;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        J.cnt->starts_done = 0;
        J.cnt->converged = 0;
        J.cnt->nonconverged = 0;
        J.cnt->sweeps_total = 0;
    }
}

// Histograms of the minima (the distribution studies of Sec. IV.B): first the
// lowest F among the counted copies (IEEE bits of F >= 0 order like the
// values), then one atomic add per counted copy into its bin.
__global__ void hist_min_kernel(const GcCopyRec *__restrict__ copies, const unsigned long long *n_copies,
                                uint32_t require_flags, unsigned long long *fmin_bits)
{
    const uint64_t n = *n_copies;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (uint64_t)gridDim.x * blockDim.x)
        if ((copies[c].flags & require_flags) == require_flags)
            atomicMin(fmin_bits, (unsigned long long)__double_as_longlong(copies[c].F));
}

__global__ void hist_kernel(const GcCopyRec *__restrict__ copies, const unsigned long long *n_copies, double dV,
                            int quantity, int weight_hits, uint32_t require_flags, double lo, double hi, int n_bins,
                            unsigned long long *counts, const unsigned long long *fmin_bits)
{
    const uint64_t n = *n_copies;
    const double Fg = __longlong_as_double((long long)*fmin_bits);
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (uint64_t)gridDim.x * blockDim.x) {
        const GcCopyRec r = copies[c];
        if ((r.flags & require_flags) != require_flags) continue;
        const double v = quantity == 0 ? r.F / dV : (r.F - Fg) / Fg;
        int b;
        if (!(v >= lo)) b = 0;
        else if (!(v < hi)) b = n_bins + 1;
        else b = 1 + min(n_bins - 1, (int)((v - lo) / (hi - lo) * (double)n_bins));
        atomicAdd(&counts[b], weight_hits ? (unsigned long long)r.hits : 1ULL);
    }
}

// Bytes carried in a kernel argument and written to device memory: lets a
// caller enqueue descriptors without host staging memory.
constexpr size_t kStoreMax = 2048;
struct StoreBytes {
    unsigned char b[kStoreMax];
};

__global__ void store_kernel(StoreBytes v, uint32_t n, unsigned char *dst)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = v.b[i];
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

size_t gc_post_lds_bytes(int d, int V, int keys, int lmax)
{
    // the link angles (key pass), or the state and the tridiagonal (filter)
    if (keys) return 4 * (size_t)d * V;
    const size_t l = (size_t)std::min(std::min(lmax, GC_LMAX), V);
    return 16 * (size_t)V + 16 * l;
}

void gc_post_shape(int V, int *block, int *sp, int *wreg)
{
    // up to 6 sites per thread with the link weights in registers; the
    // largest lattices keep them in global memory
    static const int shapes[][4] = {{64, 64, 1, 1},     {128, 64, 2, 1},    {256, 64, 4, 1},
                                    {512, 128, 4, 1},   {1024, 256, 4, 1},  {1536, 256, 6, 1},
                                    {4096, 512, 8, 0}};
    for (const auto &t : shapes)
        if (V <= t[0]) {
            *block = t[1];
            *sp = t[2];
            *wreg = t[3];
            return;
        }
    *block = 0;
    *sp = 0;
    *wreg = 0;
}

#define GC_POST_DISPATCH(FN, ...)                                                                         \
    if (block == 64 && sp == 1 && wreg) return keys ? FN<64, 1, true, true>(__VA_ARGS__)                 \
                                                    : FN<64, 1, true, false>(__VA_ARGS__);               \
    if (block == 64 && sp == 2 && wreg) return keys ? FN<64, 2, true, true>(__VA_ARGS__)                 \
                                                    : FN<64, 2, true, false>(__VA_ARGS__);               \
    if (block == 64 && sp == 4 && wreg) return keys ? FN<64, 4, true, true>(__VA_ARGS__)                 \
                                                    : FN<64, 4, true, false>(__VA_ARGS__);               \
    if (block == 128 && sp == 4 && wreg) return keys ? FN<128, 4, true, true>(__VA_ARGS__)               \
                                                     : FN<128, 4, true, false>(__VA_ARGS__);             \
    if (block == 256 && sp == 4 && wreg) return keys ? FN<256, 4, true, true>(__VA_ARGS__)               \
                                                     : FN<256, 4, true, false>(__VA_ARGS__);             \
    if (block == 256 && sp == 6 && wreg) return keys ? FN<256, 6, true, true>(__VA_ARGS__)               \
                                                     : FN<256, 6, true, false>(__VA_ARGS__);             \
    if (block == 512 && sp == 8 && !wreg) return keys ? FN<512, 8, false, true>(__VA_ARGS__)             \
                                                      : FN<512, 8, false, false>(__VA_ARGS__);           \
    return hipErrorInvalidValue;

template <int B, int SP, bool WREG, bool KEYS>
static hipError_t post_occ_t(size_t lds, int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, post_kernel<B, SP, WREG, KEYS>, B, lds);
}

template <int B, int SP, bool WREG, bool KEYS>
static hipError_t post_launch_t(const GcJobDev *jobs, int n_jobs, const uint64_t *prefix, unsigned long long *next,
                                uint64_t total, double *wbuf, uint64_t wstride, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((post_kernel<B, SP, WREG, KEYS>), dim3(grid), dim3(B), lds, s, jobs, n_jobs, prefix, next,
                       total, wbuf, wstride);
    return hipGetLastError();
}

hipError_t gc_post_occupancy(int block, int sp, int wreg, int keys, size_t lds_bytes, int *blocks_per_cu)
{
    GC_POST_DISPATCH(post_occ_t, lds_bytes, blocks_per_cu)
}

hipError_t gc_launch_post(int block, int sp, int wreg, int keys, const GcJobDev *jobs, int n_jobs,
                          const uint64_t *prefix, unsigned long long *next, uint64_t total, double *wbuf,
                          uint64_t wstride, int grid, size_t lds_bytes, hipStream_t s)
{
    GC_POST_DISPATCH(post_launch_t, jobs, n_jobs, prefix, next, total, wbuf, wstride, grid, lds_bytes, s)
}

// Line-segment filter shapes: S sites per thread along direction 0 (a
// divisor of N_0), the fewest wavefronts, then the shortest segment.
static const int kSegs[] = {1, 2, 3, 4, 5, 6, 7, 8, 10};

int gc_lanczos_shape(int d, const int *ext, int V, int *block, int *seg)
{
    (void)d;
    const int N0 = ext[0];
    int best_w = 1 << 30, best_s = 0;
    for (int S : kSegs) {
        if (N0 % S) continue;
        const int w = (V / S + 63) / 64;
        if (w > 8) continue;
        if (w < best_w) {
            best_w = w;
            best_s = S;
        }
    }
    if (!best_s) return 0;
    *seg = best_s;
    *block = best_w <= 1 ? 64 : best_w <= 2 ? 128 : best_w <= 4 ? 256 : 512;
    return 1;
}

int gc_lanczos_form(int N0, int S, int V, int block)
{
    return (S == N0 ? 1 : 0) | (V / S <= 7 * block / 8 ? 2 : 0);
}

size_t gc_lanczos_lds_bytes(int d, int N0, int S, int V, int lmax, int block)
{
    const int nw = (S == N0) ? d - 1 : d;
    const int P = (gc_lanczos_form(N0, S, V, block) & 2) ? 7 * block / 8 : block;
    const size_t l = (size_t)std::min(std::min(lmax, GC_LMAX), V);
    return 8 * (size_t)(1 + nw) * S * P + 16 * l;
}

#define GC_LANCZOS_DECLARE_DIM(D)                                                                         \
    hipError_t gc_lanczos_occupancy_d##D(int block, int seg, int form, size_t lds_bytes,                  \
                                         int *blocks_per_cu);                                             \
    hipError_t gc_launch_lanczos_d##D(int block, int seg, int form, const GcJobDev *jobs, int n_jobs,     \
                                      unsigned long long *next, int grid, size_t lds_bytes, hipStream_t s);
GC_LANCZOS_DECLARE_DIM(1)
GC_LANCZOS_DECLARE_DIM(2)
GC_LANCZOS_DECLARE_DIM(3)
GC_LANCZOS_DECLARE_DIM(4)

hipError_t gc_lanczos_occupancy(int d, int block, int seg, int form, size_t lds_bytes, int *blocks_per_cu)
{
    switch (d) {
    case 1: return gc_lanczos_occupancy_d1(block, seg, form, lds_bytes, blocks_per_cu);
    case 2: return gc_lanczos_occupancy_d2(block, seg, form, lds_bytes, blocks_per_cu);
    case 3: return gc_lanczos_occupancy_d3(block, seg, form, lds_bytes, blocks_per_cu);
    case 4: return gc_lanczos_occupancy_d4(block, seg, form, lds_bytes, blocks_per_cu);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gc_launch_lanczos(int d, int block, int seg, int form, const GcJobDev *jobs, int n_jobs,
                             unsigned long long *next, int grid, size_t lds_bytes, hipStream_t s)
{
    switch (d) {
    case 1: return gc_launch_lanczos_d1(block, seg, form, jobs, n_jobs, next, grid, lds_bytes, s);
    case 2: return gc_launch_lanczos_d2(block, seg, form, jobs, n_jobs, next, grid, lds_bytes, s);
    case 3: return gc_launch_lanczos_d3(block, seg, form, jobs, n_jobs, next, grid, lds_bytes, s);
    case 4: return gc_launch_lanczos_d4(block, seg, form, jobs, n_jobs, next, grid, lds_bytes, s);
    default: return hipErrorInvalidValue;
    }
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
        const uint32_t nblk = (uint32_t)((J.table_mask + 1 + 255) / 256);
        hipLaunchKernelGGL(count_kernel, dim3(nblk), dim3(256), 0, s, J);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, J, nblk);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(scatter_kernel, dim3(nblk), dim3(256), 0, s, J);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The paper's value-based count (Sec. III): distinct trunc(x * 1e8) over the
// converged starts.  Each converged start of [lo, hi) sets its value's bit;
// an atomic OR tells whether the bit was new, and new bits add to *count, so
// after the launch *count holds the distinct values among all starts marked
// so far.  The block-stride loop runs the same number of iterations on every
// lane of a block, so the ballot sees the whole wavefront.
__global__ void __launch_bounds__(256) paper_mark_kernel(const GcStartRec *__restrict__ rec, uint64_t lo, uint64_t hi,
                                                         uint32_t *bits, unsigned long long *count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = lo + (uint64_t)blockIdx.x * blockDim.x; base < hi; base += stride) {
        const uint64_t s = base + threadIdx.x;
        bool fresh = false;
        if (s < hi && rec[s].status == GC_ST_CONVERGED) {
            const uint32_t X = rec[s].paper_X;
            if (X < GC_PAPER_VALUES) {
                const uint32_t b = 1u << (X & 31);
                const uint32_t old =
                    __hip_atomic_fetch_or(&bits[X >> 5], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                fresh = !(old & b);
            }
        }
        const uint64_t n = (uint64_t)__popcll(__ballot(fresh));
        if ((threadIdx.x & 63) == 0 && n)
            __hip_atomic_fetch_add(count, (unsigned long long)n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t gc_launch_paper_mark(const GcStartRec *rec, uint64_t lo, uint64_t hi, uint32_t *bits,
                                unsigned long long *count, hipStream_t s)
{
    if (hi <= lo) return hipSuccess;
    const uint64_t need = (hi - lo + 255) / 256;
    const uint64_t blocks = need < 65536 ? need : 65536;
    hipLaunchKernelGGL(paper_mark_kernel, dim3((unsigned)blocks), dim3(256), 0, s, rec, lo, hi, bits, count);
    return hipGetLastError();
}

hipError_t gc_launch_orbit_random(double *phi, int64_t n_links, uint64_t seed, uint64_t orbit_index, hipStream_t s)
{
    const int64_t blocks4 = (n_links + 3) / 4;
    hipLaunchKernelGGL(orbit_random_kernel, dim3((unsigned)((blocks4 + 255) / 256)), dim3(256), 0, s, phi, n_links,
                       seed, orbit_index);
    return hipGetLastError();
}

hipError_t gc_launch_sync(const GcJobDev *jobs_host, int n_jobs, hipStream_t s)
{
    for (int j = 0; j < n_jobs; ++j) {
        const GcJobDev &J = jobs_host[j];
        const uint64_t nb = (J.n_starts + J.sync_batch - 1) / J.sync_batch;
        hipLaunchKernelGGL(sync_kernel, dim3(grid_for(nb)), dim3(256), 0, s, J);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gc_launch_store(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    for (size_t off = 0; off < bytes; off += kStoreMax) {
        StoreBytes v;
        const size_t n = bytes - off < kStoreMax ? bytes - off : kStoreMax;
        memcpy(v.b, (const unsigned char *)src + off, n);
        hipLaunchKernelGGL(store_kernel, dim3(1), dim3(256), 0, s, v, (uint32_t)n, (unsigned char *)dst + off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gc_launch_histogram(const GcCopyRec *copies, const unsigned long long *n_copies, double dV, int quantity,
                               int weight_hits, uint32_t require_flags, double lo, double hi, int n_bins,
                               unsigned long long *counts, unsigned long long *fmin_bits, hipStream_t s)
{
    hipLaunchKernelGGL(hist_min_kernel, dim3(256), dim3(256), 0, s, copies, n_copies, require_flags, fmin_bits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hist_kernel, dim3(256), dim3(256), 0, s, copies, n_copies, dV, quantity, weight_hits,
                       require_flags, lo, hi, n_bins, counts, fmin_bits);
    return hipGetLastError();
}

hipError_t gc_launch_zero_u64(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
