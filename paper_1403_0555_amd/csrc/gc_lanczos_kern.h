// FP filter in the line-segment layout (the fast filter kernel), templated
// on the lattice dimension and instantiated per dimension in
// gc_lanczos1.hip .. gc_lanczos4.hip.
#pragma once

#include "gc_filter.h"

namespace {

// The Ritz value of a check, computed by the first wavefront alone (a
// 65-section per round: a quarter of the vector work of the whole
// workgroup's multisection for one more round at most) and handed to the
// others through LDS.  The workgroup synchronises before (the tridiagonal is
// complete in LDS) and after.
template <int B>
__device__ double ritz_wave0(lds_cdouble *alpha, lds_cdouble *beta2, int k, double glo, double ghi, double prev,
                             double prev_step, int *ired, int &iph, bool final, double &hi_out, double *share)
{
    if (B > 64) __syncthreads();
    else wave_sync();
    double theta = 0.0, hi = 0.0;
    if (B == 64 || threadIdx.x < 64) {
        theta = ritz_min<64>(alpha, beta2, k, glo, ghi, prev, prev_step, ired, iph, kRitzTol, final, hi);
        if (B > 64 && threadIdx.x == 0) {
            share[0] = theta;
            share[1] = hi;
        }
    }
    if (B > 64) {
        __syncthreads();
        theta = share[0];
        hi = share[1];
    }
    hi_out = hi;
    return theta;
}

// FP filter in the line-segment layout, one workgroup of B threads per copy
// of the compacted tables (at the copy's representative start): thread t
// owns S consecutive sites along direction 0 (x_0 runs fastest, so they are
// consecutive site indices), segment t % (N_0/S) of line t / (N_0/S).  The
// Lanczos vector u of the own sites, q_{j-1} and M u stay in registers, and
// so do the direction-0 link weights; direction-0 neighbours inside the
// segment are the thread's own entries.  LDS holds u for the other
// threads, the forward link weights of directions 1..d-1 (and of direction
// 0 when a line has several segments), S P doubles each, and the
// tridiagonal.  LDS arrays are segment-major with a compile-time stride P
// (B, or 7B/8 when the launch's T = V/S threads fit in it): the k-th site
// of thread t's segment sits at k P + t, so the threads of a wavefront
// touch consecutive doubles, a neighbour in direction mu >= 1 (the same k
// of another segment) sits at a constant thread offset, and every site's
// address is a per-thread base plus a compile-time offset.  FORM bit 0:
// the segments are whole lines (S == N0); bit 1: P = 7B/8.  The iteration is
// post_kernel's: one reduction per iteration, the same formulas per site.
template <int B, int S, int D, int FORM>
__global__ __launch_bounds__(B) void lanczos_kernel(const GcJobDev *__restrict__ jobs, int n_jobs,
                                                    unsigned long long *next)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[2 * 4 * (B / 64)];
    __shared__ int ired[2 * (B / 64)];
    __shared__ double ritz[2];
    __shared__ unsigned long long claim;
    int rph = 0, iph = 0;   // halves of the reduction scratch in use
    for (;;) {
        const int tid = (int)threadIdx.x + opaque_zero();
        if (tid == 0) claim = atomicAdd(next, 1ULL);
        __syncthreads();
        const uint64_t s = uniform((uint64_t)claim);
        __syncthreads();
        int jn;
        uint64_t c;
        copy_item(jobs, n_jobs, s, jn, c);
        jn = uniform(jn);
        if (jn < 0) break;
        const GcJobDev &J = jobs[jn];
        const GcOrbitDev &O = J.orb;
        const int V = O.V, N0 = O.ext[0];
        constexpr int d = D;   // the jobs of a launch share the dimension
        const uint64_t local = J.copies[c].rep_start - J.first_start;
        const int nseg = N0 / S;
        const bool act = tid < V / S;
        const int line = act ? tid / nseg : 0, o = act ? (tid % nseg) * S : 0;
        const int i0 = line * N0 + o;
        constexpr bool whole = (FORM & 1) != 0;   // the segment is a whole line (S == N0)
        constexpr int P = (FORM & 2) ? 7 * B / 8 : B;   // stride of the segment-major arrays (>= V/S)
        const int nw = whole ? d - 1 : d;   // weight arrays in LDS
        const int w0off = whole ? -1 : 0;   // LDS array of direction mu: mu + w0off
        constexpr int A = S * P;            // doubles per LDS array
        lds_ptr<double> u = as_lds(reinterpret_cast<double *>(smem));
        lds_ptr<double> wl = u + A;
        const int lmax = min(min(J.lanczos_max, GC_LMAX), V);
        lds_ptr<double> alpha = wl + (size_t)nw * A;
        lds_ptr<double> beta2 = alpha + lmax;

        // own link weights w = Re(conj(g_i) U_{i,mu} g_{i+mu}) from the
        // representative's state in global memory: direction 0 into
        // registers, the others into LDS
        glb_ptr<const dbl2> src = as_global(reinterpret_cast<const dbl2 *>(J.states + local * (uint64_t)V));
        glb_ptr<const dbl2> Ug = as_global(reinterpret_cast<const dbl2 *>(O.U64));
        double w0[S];
        // thread offsets of the neighbours in directions >= 1 (the same for
        // every own site: site offsets, multiples of N0, divided by S)
        int df[GC_MAXD], db[GC_MAXD];
#pragma unroll
        for (int mu = 0; mu < GC_MAXD; ++mu) {
            df[mu] = 0;
            db[mu] = 0;
            if (act && mu > 0 && mu < d) {
                df[mu] = ((int)O.nbr[mu * V + i0] - i0) / S;
                db[mu] = ((int)O.nbr[(d + mu) * V + i0] - i0) / S;
            }
        }
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int i = i0 + k;
            w0[k] = 0.0;
            if (act) {
                const dbl2 gi = src[i];
#pragma unroll
                for (int mu = 0; mu < GC_MAXD; ++mu) {
                    if (mu < d) {
                        const dbl2 gf = src[O.nbr[mu * V + i]];
                        const dbl2 uu = Ug[mu * V + i];
                        const double tr = uu.x * gf.x - uu.y * gf.y, ti = uu.x * gf.y + uu.y * gf.x;
                        const double ur = gi.x * tr + gi.y * ti;
                        if (mu == 0) w0[k] = ur;
                        if (mu + w0off >= 0) wl[(mu + w0off) * A + k * P + tid] = ur;
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        double uo[S], qp[S], mv[S];
        double sums[1] = {0.0};
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int i = i0 + k;
            qp[k] = 0.0;
            uo[k] = 0.0;
            mv[k] = 0.0;
            if (act) {
                const double x = (double)(mix64((uint64_t)i + 0x5851F42D4C957F2DULL) >> 11) * 0x1.0p-53 - 0.5;
                uo[k] = x;
                sums[0] += x;
            }
        }
        wg_sum_n<B, 1>(sums, red, rph);
        const double mean = sums[0] / (double)V;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            if (act) {
                uo[k] -= mean;
                u[k * P + tid] = uo[k];
            }
        }
        const double sigma = 4.0 * d + 1.0;
        const double sigma_v = sigma / (double)V;   // the weight of the projector on the constant vector
        double theta = INFINITY, theta_old = INFINITY, theta_step = 1.0;
        double rows_lo = INFINITY, rows_hi = -INFINITY;   // Gershgorin bounds of the complete rows
        double a_prev = 0.0, b_prev2 = 0.0;                // alpha_{j-1}, beta_{j-2}
        int next_check = kFirstCheck;                      // iteration count of the next Ritz check
        int it = 0;
        bool conv = false;
        // the neighbours across the ends of a segment that is not a whole
        // line: the first site of the next segment, the last of the previous
        const int ia = line * nseg + ((o + S) % N0) / S;
        const int ib = (S - 1) * P + line * nseg + ((o + N0 - 1) % N0) / S;
        // byte offsets from u of the four values a site reads per direction
        // mu >= 1 (fixed for the copy): the own forward weight (aw), the
        // forward neighbour's u (af), the backward neighbour's weight (bw)
        // and u (bu); the k-th site adds a compile-time offset.  Each is its
        // own register, opaque to the compiler: two loads from one register
        // would be paired into a ds_read2st64, whose two addresses, a
        // multiple of 512 bytes apart, fall in the same LDS bank.
        lds_ptr<const unsigned char> ubase = (lds_ptr<const unsigned char>)u;
        uint32_t aw[GC_MAXD], af[GC_MAXD], bw[GC_MAXD], bu[GC_MAXD];
#pragma unroll
        for (int mu = 0; mu < GC_MAXD; ++mu) {
            const uint32_t warr = 8u * (uint32_t)((1 + mu + w0off) * A);   // the weight array of mu
            aw[mu] = warr + 8u * (uint32_t)tid;
            af[mu] = 8u * (uint32_t)(tid + df[mu]);
            bw[mu] = warr + 8u * (uint32_t)(tid + db[mu]);
            bu[mu] = 8u * (uint32_t)(tid + db[mu]);
            if (mu > 0 && mu < d) asm volatile("" : "+v"(aw[mu]), "+v"(af[mu]), "+v"(bw[mu]), "+v"(bu[mu]));
        }
        // the diagonal of M at the own sites, the sum of their 2d link
        // weights, once per copy (M u)_i = diag_i u_i - sum_nb w u_nb
        if (B > 64) __syncthreads();   // the weights complete in LDS
        else wave_sync();
        double dg[S];
        {
            const double wbe0 = whole ? w0[S - 1] : wl[ib];
#pragma unroll
            for (int k = 0; k < S; ++k) {
                double a = w0[k] + ((k > 0) ? w0[k - 1] : wbe0);
#pragma unroll
                for (int mu = 1; mu < GC_MAXD; ++mu)
                    if (mu < d) {
                        lds_ptr<const double> wm = wl + (mu + w0off) * A + k * P;
                        a += wm[tid] + wm[tid + db[mu]];
                    }
                dg[k] = act ? a : 0.0;
            }
        }
        for (it = 0; it < lmax; ++it) {
            if (B > 64) __syncthreads();   // u and the weights complete in LDS
            else wave_sync();
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
            if (act) {
                double ua, ub, wbe;
                if constexpr (whole) {
                    ua = uo[0];
                    ub = uo[S - 1];
                    wbe = w0[S - 1];
                } else {
                    ua = u[ia];
                    ub = u[ib];
                    wbe = wl[ib];
                }
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    const uint32_t kb = 8u * (uint32_t)(k * P);
                    const double ui = uo[k];
                    // direction 0: neighbours and weights of the own segment
                    const double uf = (k + 1 < S) ? uo[k + 1] : ua;
                    const double ubk = (k > 0) ? uo[k - 1] : ub;
                    const double wb0 = (k > 0) ? w0[k - 1] : wbe;
                    double m = dg[k] * ui;
                    m = fma(-w0[k], uf, m);
                    m = fma(-wb0, ubk, m);
#pragma unroll
                    for (int mu = 1; mu < GC_MAXD; ++mu)
                        if (mu < d) {
                            lds_ptr<const unsigned char> b8 = ubase + kb;
                            const double wf_ = *(lds_ptr<const double>)(b8 + aw[mu]);
                            const double uf_ = *(lds_ptr<const double>)(b8 + af[mu]);
                            const double wb_ = *(lds_ptr<const double>)(b8 + bw[mu]);
                            const double ub_ = *(lds_ptr<const double>)(b8 + bu[mu]);
                            m = fma(-wf_, uf_, m);
                            m = fma(-wb_, ub_, m);
                        }
                    mv[k] = m;
                    s4[0] += ui * ui;
                    s4[1] += ui * m;
                    s4[2] += ui;
                    s4[3] += ui * qp[k];
                    // one site at a time: bounds the loads in flight
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            wg_sum_n<B, 4>(s4, red, rph);
            // 1/|u| from the reciprocal square root, no division on the
            // iteration's dependency chain (a vanishing |u| gives bt = 0)
            const double inv = rsq(fmax(s4[0], 1e-300));
            const double bt = s4[0] * inv;
            const double bp = it > 0 ? bt : 0.0;      // beta_{j-1} (the start vector's norm is not in T)
            if (it > 0) {
                if (tid == 0) beta2[it - 1] = s4[0];
                rows_lo = fmin(rows_lo, a_prev - b_prev2 - bt);
                rows_hi = fmax(rows_hi, a_prev + b_prev2 + bt);
                if (bt <= 1e-13 * sigma) {
                    // the Krylov space is exhausted: T of it rows is exact
                    double theta_hi;
                    theta = ritz_wave0<B>(alpha, beta2, it, rows_lo, rows_hi, theta_old, theta_step, ired, iph, true,
                                          theta_hi, ritz);
                    conv = true;
                    break;
                }
            }
            const double sq = s4[2] * inv;
            const double shift = sigma_v * sq;
            const double a_j = s4[1] * inv * inv + shift * sq - bp * (s4[3] * inv);
            if (tid == 0) alpha[it] = a_j;
            if (act) {
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    const double q = uo[k] * inv;
                    const double r = mv[k] * inv + shift - bp * qp[k] - a_j * q;
                    qp[k] = q;
                    uo[k] = r;
                    u[k * P + tid] = r;
                }
            }
            if (it + 1 >= next_check || it + 1 == lmax) {
                const bool final = it + 1 == lmax;
                double theta_hi;
                theta = ritz_wave0<B>(alpha, beta2, it + 1, fmin(rows_lo, a_j - bp), fmax(rows_hi, a_j + bp),
                                      theta_old, theta_step, ired, iph, final, theta_hi, ritz);
                const double tol = kRitzTol * fmax(1.0, fabs(theta));
                const double change = theta_old - theta;
                if (fabs(change) <= tol) {
                    conv = true;
                    ++it;
                    break;
                }
                const int gap = check_gap(change, tol);
                next_check = it + 1 + gap;
                if (theta_old < INFINITY) theta_step = change;
                theta_old = theta_hi;
            }
            b_prev2 = bp;
            a_prev = a_j;
        }
        uint32_t flags = region_flags(theta, J.lambda_tol);
        if (!conv) flags |= GC_F_LANCZOS_CAP;
        if (tid == 0) {
            write_filter(J, c, local, theta, flags, (uint32_t)it);
            atomicAdd(&J.cnt->lanczos_runs, 1ULL);
        }
        __syncthreads();
    }
}

}  // namespace

// Entry points of one lattice dimension D (gc_lanczosD.hip): occupancy and
// launch of lanczos_kernel<B, S, D, FORM> for the shapes gc_lanczos_shape
// and gc_lanczos_form pick.
#define GC_LANCZOS_F(FN, B, S, D, ...)                                                                    \
    switch (form) {                                                                                       \
    case 0: return FN<B, S, D, 0>(__VA_ARGS__);                                                           \
    case 1: return FN<B, S, D, 1>(__VA_ARGS__);                                                           \
    case 2: return FN<B, S, D, 2>(__VA_ARGS__);                                                           \
    case 3: return FN<B, S, D, 3>(__VA_ARGS__);                                                           \
    default: return hipErrorInvalidValue;                                                                 \
    }
#define GC_LANCZOS_SEG(FN, B, D, ...)                                                                     \
    switch (seg) {                                                                                        \
    case 1: GC_LANCZOS_F(FN, B, 1, D, __VA_ARGS__)                                                        \
    case 2: GC_LANCZOS_F(FN, B, 2, D, __VA_ARGS__)                                                        \
    case 3: GC_LANCZOS_F(FN, B, 3, D, __VA_ARGS__)                                                        \
    case 4: GC_LANCZOS_F(FN, B, 4, D, __VA_ARGS__)                                                        \
    case 5: GC_LANCZOS_F(FN, B, 5, D, __VA_ARGS__)                                                        \
    case 6: GC_LANCZOS_F(FN, B, 6, D, __VA_ARGS__)                                                        \
    case 7: GC_LANCZOS_F(FN, B, 7, D, __VA_ARGS__)                                                        \
    case 8: GC_LANCZOS_F(FN, B, 8, D, __VA_ARGS__)                                                        \
    case 10: GC_LANCZOS_F(FN, B, 10, D, __VA_ARGS__)                                                      \
    default: return hipErrorInvalidValue;                                                                 \
    }
#define GC_LANCZOS_DISPATCH(FN, D, ...)                                                                   \
    switch (block) {                                                                                      \
    case 64: GC_LANCZOS_SEG(FN, 64, D, __VA_ARGS__)                                                       \
    case 128: GC_LANCZOS_SEG(FN, 128, D, __VA_ARGS__)                                                     \
    case 256: GC_LANCZOS_SEG(FN, 256, D, __VA_ARGS__)                                                     \
    case 512: GC_LANCZOS_SEG(FN, 512, D, __VA_ARGS__)                                                     \
    default: return hipErrorInvalidValue;                                                                 \
    }

template <int B, int S, int D, int FORM>
static hipError_t lanczos_occ_t(size_t lds, int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, lanczos_kernel<B, S, D, FORM>, B, lds);
}

template <int B, int S, int D, int FORM>
static hipError_t lanczos_launch_t(const GcJobDev *jobs, int n_jobs, unsigned long long *next, int grid, size_t lds,
                                   hipStream_t s)
{
    hipLaunchKernelGGL((lanczos_kernel<B, S, D, FORM>), dim3(grid), dim3(B), lds, s, jobs, n_jobs, next);
    return hipGetLastError();
}

// form: gc_lanczos_form's value, the same for every job of the launch
#define GC_LANCZOS_DEFINE_DIM(D)                                                                          \
    hipError_t gc_lanczos_occupancy_d##D(int block, int seg, int form, size_t lds_bytes,                  \
                                         int *blocks_per_cu)                                              \
    {                                                                                                     \
        GC_LANCZOS_DISPATCH(lanczos_occ_t, D, lds_bytes, blocks_per_cu)                                   \
    }                                                                                                     \
    hipError_t gc_launch_lanczos_d##D(int block, int seg, int form, const GcJobDev *jobs, int n_jobs,     \
                                      unsigned long long *next, int grid, size_t lds_bytes, hipStream_t s)  \
    {                                                                                                     \
        GC_LANCZOS_DISPATCH(lanczos_launch_t, D, jobs, n_jobs, next, grid, lds_bytes, s)                  \
    }
