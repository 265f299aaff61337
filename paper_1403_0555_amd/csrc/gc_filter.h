// Device helpers of the FP filter shared by the post kernel (gc_post.hip)
// and the line-segment Lanczos kernels (gc_lanczos_kern.h): workgroup
// reductions, the Sturm-sequence Ritz value of the Lanczos tridiagonal, the
// first-region flags and the bookkeeping of a filtered copy.
#pragma once

#include "gc_common.h"

namespace {

using namespace gc;

// Workgroup reductions over B threads: wave reductions, then the waves'
// partials combined in a fixed order.  Every thread returns the result.
// Successive calls on one scratch array alternate between its two halves
// (ph toggles), so a call needs a single barrier: a half is rewritten only
// after every wave has passed the barrier of the call in between, and so has
// finished reading it.
template <int B, int N>
__device__ __forceinline__ void wg_sum_n(double (&v)[N], double *red, int &ph)
{
    wave_sum_n<N>(v);
    if (B > 64) {
        double *r = red + ph * (4 * (B / 64));
        ph ^= 1;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int n = 0; n < N; ++n) r[n * (B / 64) + (threadIdx.x >> 6)] = v[n];
        }
        __syncthreads();
#pragma unroll
        for (int n = 0; n < N; ++n) {
            double t = r[n * (B / 64)];
#pragma unroll
            for (int w = 1; w < B / 64; ++w) t += r[n * (B / 64) + w];
            v[n] = t;
        }
    }
}

template <int B>
__device__ __forceinline__ uint64_t wg_sum_u64(uint64_t v, uint64_t *red, int &ph)
{
    v = wave_sum_u64(v);
    if (B > 64) {
        uint64_t *r = red + ph * (B / 64);
        ph ^= 1;
        if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = v;
        __syncthreads();
        uint64_t t = r[0];
#pragma unroll
        for (int w = 1; w < B / 64; ++w) t += r[w];
        v = t;
    }
    return v;
}

template <int B>
__device__ __forceinline__ int wg_min_int(int v, int *red, int &ph)
{
    v = wave_min_int(v);
    if (B > 64) {
        int *r = red + ph * (B / 64);
        ph ^= 1;
        if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = v;
        __syncthreads();
        int t = r[0];
#pragma unroll
        for (int w = 1; w < B / 64; ++w) t = min(t, r[w]);
        v = t;
    }
    return v;
}

typedef __attribute__((address_space(3))) const double lds_cdouble;

// Number of eigenvalues of the k x k tridiagonal below x: the sign changes
// of the Sturm sequence p_0 = 1, p_j = det(T_j - x) = (alpha_j - x) p_{j-1}
// - beta_{j-1}^2 p_{j-2}, counted from the sign bits.  An exact zero p_j
// counts as positive: the next term is then -beta_j^2 p_{j-1}, of the sign
// opposite to p_{j-1}, so the two steps around the zero hold exactly one
// sign change, as under the usual convention (a vanishing term takes the
// sign opposite to its predecessor); every beta_j of the run is positive
// (it stops before a vanishing one).  Division- and branch-free: one
// dependent FMA per step.  The pair (p_{j-1}, p_j) is rescaled by a power of
// two after every four rows, which keeps it in range and leaves every sign
// unchanged.
__device__ __forceinline__ int sign_change(double a, double b)
{
    return (int)(((uint64_t)__double_as_longlong(a) ^ (uint64_t)__double_as_longlong(b)) >> 63);
}

__device__ __forceinline__ void sturm_step(double a, double b2, double x, double &p0, double &p1, int &cnt)
{
    const double p2 = fma(a - x, p1, -b2 * p0);
    cnt += sign_change(p2, p1);
    p0 = p1;
    p1 = p2;
}

__device__ int sturm_count(lds_cdouble *alpha, lds_cdouble *beta2, int k, double x)
{
    double p0 = 1.0, p1 = alpha[0] - x;
    int cnt = sign_change(p1, 1.0);
    int j = 1;
    for (; j + 4 <= k; j += 4) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = alpha[j + u];
            b[u] = beta2[j + u - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) sturm_step(a[u], b[u], x, p0, p1, cnt);
        int e;
        (void)frexp(p1, &e);
        p0 = ldexp(p0, -e);
        p1 = ldexp(p1, -e);
    }
    for (; j < k; ++j) sturm_step(alpha[j], beta2[j - 1], x, p0, p1, cnt);
    return cnt;
}

// Smallest eigenvalue of the tridiagonal by (B+1)-section inside [lo, hi]
// (count(lo) = 0, count(hi) >= 1), to a bracket of 1e-15 max(1, |theta|)
// when final, else of tol_rel / 100 of that (the convergence test compares
// values at tol_rel, and the value it accepts is this one, so its bracket
// error stays a hundredth of the test's tolerance).  Unless final, the
// search stops early when the eigenvalue lies more than
// 1e6 tol_rel max(1, |theta|) below prev (the previous check's upper bound)
// and the bracket is small against that distance: the convergence test then
// fails whatever the remaining digits are.  hi_out receives the final upper
// end, a guaranteed upper bound.
template <int B>
__device__ double tridiag_min_eig(lds_cdouble *alpha, lds_cdouble *beta2, int k, double lo, double hi, int *ired,
                                  int &iph, double prev, double tol_rel, bool final, double &hi_out)
{
    const double width = final ? 1e-15 : 1e-2 * tol_rel;
    for (int round = 0; round < 24; ++round) {
        if (hi - lo <= width * fmax(1.0, fabs(hi))) break;
        if (!final) {
            const double gap = prev - hi, scale = fmax(1.0, fabs(hi));
            const bool fails = gap > 1e6 * tol_rel * scale;   // far from converging
            const double need = (prev < INFINITY) ? 0.05 * gap : 1e-4 * scale;
            if (fails && hi - lo <= need) break;
        }
        const double step = (hi - lo) / (double)(B + 1);
        const double x = lo + step * (double)(threadIdx.x + 1);
        const int first = wg_min_int<B>(sturm_count(alpha, beta2, k, x) >= 1 ? (int)threadIdx.x : B, ired, iph);
        const double nlo = (first == 0) ? lo : lo + step * (double)first;
        const double nhi = (first == B) ? hi : lo + step * (double)(first + 1);
        lo = nlo;
        hi = nhi;
    }
    hi_out = hi;
    return 0.5 * (lo + hi);
}

// Smallest Ritz value of the k x k tridiagonal, inside the Gershgorin
// interval [glo, ghi].  By interlacing it never increases as k grows, so the
// previous check's upper bound prev bounds it above, and a window [bot, top]
// just below it is tried first: one round over B points that include both
// ends (x_t = bot + (top - bot) t / (B - 1)) tells at once whether the
// window holds the value (count(bot) = 0 and count(top) >= 1) and where.
template <int B>
__device__ double ritz_min(lds_cdouble *alpha, lds_cdouble *beta2, int k, double glo, double ghi, double prev,
                           double prev_step, int *ired, int &iph, double tol_rel, bool final, double &hi_out)
{
    double lo = glo - 1e-12 * (1.0 + fabs(glo));
    double hi = ghi + 1e-12 * (1.0 + fabs(ghi));
    if (prev < hi) {
        const double top = prev + 1e-12 * (1.0 + fabs(prev));
        const double bot = top - fmax(4.0 * prev_step, 1e-9 * (1.0 + fabs(prev)));
        if (bot > lo) {
            const double step = (top - bot) / (double)(B - 1);
            const double x = ((int)threadIdx.x == B - 1) ? top : bot + step * (double)threadIdx.x;
            const int first =
                wg_min_int<B>(sturm_count(alpha, beta2, k, x) >= 1 ? (int)threadIdx.x : B, ired, iph);
            if (first > 0 && first < B)
                return tridiag_min_eig<B>(alpha, beta2, k, bot + step * (double)(first - 1),
                                          (first == B - 1) ? top : bot + step * (double)first, ired, iph, prev,
                                          tol_rel, final, hi_out);
            if (first == 0) hi = bot;   // below the window: bot bounds it above
        } else if (sturm_count(alpha, beta2, k, top) >= 1) {
            hi = top;
        }
    }
    return tridiag_min_eig<B>(alpha, beta2, k, lo, hi, ired, iph, prev, tol_rel, final, hi_out);
}

// Lanczos stops when the lowest Ritz value moved by at most this relative
// amount since the previous check (at least 8 iterations earlier).  Its
// error is then of the same order, some 1e-11 in absolute terms for these
// operators, far below the region threshold (1e-6).
constexpr double kRitzTol = 1e-10;

// The checks' schedule: the first after kFirstCheck iterations, then every
// 24 while the lowest Ritz value still moves by more than 1e6 times the
// tolerance, every 16 while it moves by more than 1e3 times, else every 8
// (the value settles by about a decade per 8 iterations near the end).
constexpr int kFirstCheck = 24;
__device__ __forceinline__ int check_gap(double change, double tol)
{
    return !(change <= 1e6 * tol) ? 24 : !(change <= 1e3 * tol) ? 16 : 8;
}

__device__ uint32_t region_flags(double lam2, double tol)
{
    if (lam2 > tol) return GC_F_IN_REGION;
    if (lam2 < -tol) return GC_F_SADDLE;
    return GC_F_SINGULAR;
}

constexpr uint32_t kFilterFlags = GC_F_IN_REGION | GC_F_SINGULAR | GC_F_SADDLE | GC_F_LANCZOS_CAP;

// The filter's results: into the copy and its representative's start record.
__device__ void write_filter(const GcJobDev &J, uint64_t c, uint64_t local, double lam2, uint32_t flags, uint32_t lit)
{
    GcCopyRec &cp = J.copies[c];
    cp.lambda2 = lam2;
    cp.flags |= flags & kFilterFlags;
    cp.lanczos_iters = lit;
    GcStartRec &r = J.rec[local];
    r.lambda2 = lam2;
    r.flags = (r.flags & ~kFilterFlags) | (flags & kFilterFlags);
    r.lanczos_iters = lit;
}

// The item of a filter pass: copy s of the concatenated copy lists of the
// jobs (job order), or jn = -1 past the end.
__device__ __forceinline__ void copy_item(const GcJobDev *jobs, int n_jobs, uint64_t s, int &jn, uint64_t &c)
{
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
    c = s - base;
}

}  // namespace
