// gfx950 kernels of the Gribov-copy enumerator for compact U(1).
//
// One workgroup holds one random start at a time: its gauge transformation
// g_i = exp(i theta_i) lives in LDS for the whole solve, the orbit's link
// field and neighbour tables are read through L1/L2 (shared by every
// workgroup on the orbit), and the workgroup pulls the next start from a
// device-wide counter when its start has converged.  A start therefore never
// waits for a slower one, which removes the fixed-grid stall of the paper's
// implementation (Sec. III: the runtime of a fixed batch is set by its
// slowest sample).  Per start, in order:
//   init     theta_i by Philox4x64-10 (Sec. III) -> g_i
//   sweeps   colour c = 0..K-1, every site of colour c updated concurrently
//            (checkerboard, Sec. III) by the local maximisation of eqs.
//            (4)-(5) in the convention of eq. (3): g_i <- S_i/|S_i|, or the
//            over-relaxed g_i <- g_i N(1 + omega (z - 1)), z = conj(g_i) S_i/|S_i|
//   stop     (1/V) sum div_i^2 < eps (or max |div_i| < eps, the paper's rule)
//            with div_i = Im(conj(g_i) S_i), on the post-sweep state
//   mixed    single-precision sweeps to eps32, promote, double polish to eps64
//   observe  u_l = conj(g_i) U_l g_{i+mu}, F = sum (1 - Re u_l) (eq. (3)),
//            x = F/(dV), the paper's X = trunc(x 1e8) (Sec. III)
//   key      plaquette and line wrap numbers of a_l = arg u_l relative to
//            the orbit's raw plaquette and line sums, hashed to 128 bits
//   dedup    open-addressing insert into the orbit's copy table
//   filter   for the lowest start id of a key: Lanczos on the FP operator
//            M = B^T diag(Re u) B (the Hessian of eq. (3)) shifted by
//            sigma 11^T/V, giving lambda2, the lowest eigenvalue off the
//            constant mode (first Gribov region test)
#include "gc_internal.h"

#include <math.h>

namespace {

constexpr double kPi = 3.14159265358979311599796346854;
constexpr double kTwoPi = 6.28318530717958623199592693709;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and the angle map of the random starts
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += W0; k1 += W1;
    }
}

// fl(fl(u * 2pi) - pi), u = (r >> 11) 2^-53, with contraction switched off
// so that the product is rounded before the subtraction.
__device__ __forceinline__ double angle_of(uint64_t r)
{
#pragma clang fp contract(off)
    const double u = (double)(r >> 11) * 0x1.0p-53;
    const double t = u * kTwoPi;
    return t - kPi;
}

// arg(g conj(gl)) in (-pi, pi]; unfused so that g = gl gives exactly 0.
__device__ __forceinline__ double rel_angle(double2 g, double2 gl)
{
#pragma clang fp contract(off)
    const double im = g.y * gl.x - g.x * gl.y;
    const double re = g.x * gl.x + g.y * gl.y;
    return atan2(im, re);
}

// SplitMix64 output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Workgroup reductions (fixed butterfly + fixed cross-wave order: the result
// depends only on the block size, not on scheduling)
// ---------------------------------------------------------------------------
template <int B>
__device__ __forceinline__ double wg_sum(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int k = 1; k < B / 64; ++k) s += red[k];
    return s;
}

template <int B>
__device__ __forceinline__ double wg_max(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int k = 1; k < B / 64; ++k) s = fmax(s, red[k]);
    return s;
}

template <int B>
__device__ __forceinline__ double wg_min(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int k = 1; k < B / 64; ++k) s = fmin(s, red[k]);
    return s;
}

template <int B>
__device__ __forceinline__ uint64_t wg_sum_u64(uint64_t v, uint64_t *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t s = red[0];
#pragma unroll
    for (int k = 1; k < B / 64; ++k) s += red[k];
    return s;
}

template <int B>
__device__ __forceinline__ int wg_min_int(int v, int *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int s = red[0];
#pragma unroll
    for (int k = 1; k < B / 64; ++k) s = min(s, red[k]);
    return s;
}

// ---------------------------------------------------------------------------
// Local update, eqs. (4)-(5) in the eq. (3) convention
// ---------------------------------------------------------------------------
template <typename R> struct cvec;
template <> struct cvec<float> { using T = float2; };
template <> struct cvec<double> { using T = double2; };

__device__ __forceinline__ float rsqrt_r(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return rsqrt(x); }

template <typename R> __device__ __forceinline__ const typename cvec<R>::T *links(const GcOrbitDev &O);
template <> __device__ __forceinline__ const float2 *links<float>(const GcOrbitDev &O) { return O.U32; }
template <> __device__ __forceinline__ const double2 *links<double>(const GcOrbitDev &O) { return O.U64; }

// S_i = sum_mu [U_{i,mu} g_{i+mu} + conj(U_{i-mu,mu}) g_{i-mu}]
template <typename R>
__device__ __forceinline__ typename cvec<R>::T staple(const GcOrbitDev &O, const typename cvec<R>::T *__restrict__ U,
                                                      const typename cvec<R>::T *st, int i)
{
    const int V = O.V, d = O.d;
    R ax = 0, ay = 0;
    for (int mu = 0; mu < d; ++mu) {
        const int f = O.nbr[mu * V + i];
        const int b = O.nbr[(d + mu) * V + i];
        const typename cvec<R>::T u = U[mu * V + i];
        const typename cvec<R>::T gf = st[f];
        ax += u.x * gf.x - u.y * gf.y;
        ay += u.x * gf.y + u.y * gf.x;
        const typename cvec<R>::T v = U[mu * V + b];
        const typename cvec<R>::T gb = st[b];
        ax += v.x * gb.x + v.y * gb.y;
        ay += v.x * gb.y - v.y * gb.x;
    }
    typename cvec<R>::T s;
    s.x = ax;
    s.y = ay;
    return s;
}

// Sweeps of one precision until the stopping norm falls below eps or the
// sweep cap is hit.  Returns the status; sweeps and the final norm by ref.
template <typename R, int B>
__device__ int relax_phase(const GcJobDev &J, typename cvec<R>::T *st, double eps, uint64_t &sweeps,
                           double &D, double *red)
{
    using C = typename cvec<R>::T;
    const GcOrbitDev &O = J.orb;
    const C *__restrict__ U = links<R>(O);
    const int V = O.V, K = O.K, tid = threadIdx.x;
    const R omega = (R)J.omega;
    const bool relax = (omega == (R)1);
    const uint64_t check = J.check_every > 0 ? (uint64_t)J.check_every : 1;
    uint64_t t = 0;
    int status = GC_ST_NONCONVERGED;
    D = INFINITY;
    while (t < J.max_sweeps) {
        for (int c = 0; c < K; ++c) {
            const int lo = O.coff[c], hi = O.coff[c + 1];
            for (int p = lo + tid; p < hi; p += B) {
                const int i = O.perm[p];
                const C s = staple<R>(O, U, st, i);
                const R n2 = s.x * s.x + s.y * s.y;
                if (n2 == (R)0) continue;
                const R r = rsqrt_r(n2);
                const R hx = s.x * r, hy = s.y * r;
                C g;
                if (relax) {
                    g.x = hx;
                    g.y = hy;
                } else {
                    const C g0 = st[i];
                    const R zx = g0.x * hx + g0.y * hy;
                    const R zy = g0.x * hy - g0.y * hx;
                    R wx = (R)1 + omega * (zx - (R)1);
                    R wy = omega * zy;
                    const R rw = rsqrt_r(wx * wx + wy * wy);
                    wx *= rw;
                    wy *= rw;
                    g.x = g0.x * wx - g0.y * wy;
                    g.y = g0.x * wy + g0.y * wx;
                }
                st[i] = g;
            }
            __syncthreads();
        }
        ++t;
        if (t % check == 0 || t == J.max_sweeps) {
            double acc = 0.0;
            for (int i = tid; i < V; i += B) {
                const C s = staple<R>(O, U, st, i);
                const C g = st[i];
                const double dv = (double)(g.x * s.y - g.y * s.x);
                acc = J.stop_norm ? fmax(acc, fabs(dv)) : acc + dv * dv;
            }
            D = J.stop_norm ? wg_max<B>(acc, red) : wg_sum<B>(acc, red) / (double)V;
            if (!(D == D)) { status = GC_ST_BADNUM; break; }
            if (D < eps) { status = GC_ST_CONVERGED; break; }
        }
    }
    sweeps = t;
    return status;
}

// Smallest eigenvalue of the k x k tridiagonal (alpha, beta) by multisection
// on the Sturm count (number of eigenvalues below x from the LDL^T pivots).
template <int B>
__device__ double tridiag_min_eig(const double *alpha, const double *beta, int k, int *ired)
{
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
        // points x_t = lo + step (t + 1), t = 0..B-1; the lowest eigenvalue
        // lies between the last point with count 0 and the first with >= 1
        const double step = (hi - lo) / (double)(B + 1);
        const double x = lo + step * (double)(threadIdx.x + 1);
        int cnt = 0;
        double q = alpha[0] - x;
        if (q < 0) ++cnt;
        for (int j = 1; j < k; ++j) {
            const double qq = (q == 0.0) ? 1e-300 : q;
            q = (alpha[j] - x) - beta[j - 1] * beta[j - 1] / qq;
            if (q < 0) ++cnt;
        }
        const int first = wg_min_int<B>(cnt >= 1 ? (int)threadIdx.x : B, ired);
        const double nlo = (first == 0) ? lo : lo + step * (double)first;
        const double nhi = (first == B) ? hi : lo + step * (double)(first + 1);
        lo = nlo;
        hi = nhi;
        if (hi - lo <= 1e-15 * fmax(1.0, fabs(hi))) break;
    }
    return 0.5 * (lo + hi);
}

// Insert a key into the copy table; returns (claimed new key, lowest start so far).
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
        unsigned long long old = atomicCAS((unsigned long long *)&e->key_hi, 0ULL, (unsigned long long)key_hi);
        bool match = false;
        if (old == 0ULL) {
            __hip_atomic_store(&e->key_lo, key_lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&e->ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            claimed = true;
            match = true;
        } else if (old == key_hi) {
            // The claimer writes key_lo right after its CAS; wait for it (bounded).
            uint32_t rdy = 0;
            for (int spin = 0; spin < (1 << 22); ++spin) {
                rdy = __hip_atomic_load(&e->ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (rdy) break;
                __builtin_amdgcn_s_sleep(2);
            }
            if (!rdy) return;   // failed: counted as an error by the caller
            match = (__hip_atomic_load(&e->key_lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == key_lo);
        }
        if (match) {
            atomicAdd((unsigned long long *)&e->hits, 1ULL);
            unsigned long long prev = atomicMin((unsigned long long *)&e->first_start, (unsigned long long)sid);
            atomicMin((unsigned long long *)&e->fmin_bits, (unsigned long long)fbits);
            atomicMax((unsigned long long *)&e->fmax_bits, (unsigned long long)fbits);
            is_min = sid < prev;
            failed = false;
            return;
        }
        idx = (idx + 1) & mask;
    }
}

// ---------------------------------------------------------------------------
// The persistent solve kernel
// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(B) void solve_kernel(const GcJobDev *__restrict__ jobs, int n_jobs,
                                                  const uint64_t *__restrict__ prefix,
                                                  unsigned long long *next, uint64_t total,
                                                  const unsigned long long *total_dev,
                                                  double *scratch, uint64_t scratch_stride)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[B / 64];
    __shared__ uint64_t ured[B / 64];
    __shared__ int ired[B / 64];
    __shared__ unsigned long long claim;
    __shared__ int flag_sh[2];

    const int tid = threadIdx.x;
    double *wscr = scratch + (uint64_t)blockIdx.x * scratch_stride;
    if (total_dev) total = *total_dev;

    for (;;) {
        if (tid == 0) claim = atomicAdd(next, 1ULL);
        __syncthreads();
        const unsigned long long s = claim;
        __syncthreads();
        if (s >= total) break;
        int jn = 0;
        while (jn + 1 < n_jobs && prefix[jn + 1] <= s) ++jn;
        const GcJobDev &J = jobs[jn];
        const GcOrbitDev &O = J.orb;
        const int V = O.V, d = O.d;
        const uint64_t local = s - (prefix ? prefix[jn] : 0);
        const bool fixmode = (J.flags & GC_JOB_FIX) != 0;
        const uint64_t sid = fixmode ? J.fix[local].start : J.first_start + local;

        double2 *st64 = reinterpret_cast<double2 *>(smem);
        float2 *st32 = reinterpret_cast<float2 *>(smem + 16 * (size_t)V);
        double *lq = reinterpret_cast<double *>(smem + 16 * (size_t)V);
        double *alpha = reinterpret_cast<double *>(smem + 24 * (size_t)V);
        double *beta = alpha + GC_LMAX;

        // ---- random start (Sec. III): Philox block b covers sites 4b..4b+3
        for (int b = tid; 4 * b < V; b += B) {
            uint64_t c[4] = {(uint64_t)b, sid, O.orbit_index, 0x53ULL};
            philox4x64_10(c, J.start_seed, 1ULL);
#pragma unroll 1
            for (int k = 0; k < 4; ++k) {
                const int i = 4 * b + k;
                if (i < V) {
                    double sn, cs;
                    sincos(angle_of(c[k]), &sn, &cs);
                    if (J.precision == 1) st32[i] = make_float2((float)cs, (float)sn);
                    else st64[i] = make_double2(cs, sn);
                }
            }
        }
        __syncthreads();

        uint64_t sw32 = 0, sw64 = 0;
        double D = INFINITY;
        int status;
        bool in64 = J.precision != 1;
        if (J.precision == 1) {
            status = relax_phase<float, B>(J, st32, J.eps32, sw32, D, red);
            if (status == GC_ST_CONVERGED) {
                in64 = true;
                // promotion: g64 = normalise((double) g32)
                for (int i = tid; i < V; i += B) {
                    const float2 g = st32[i];
                    const double xr = (double)g.x, xi = (double)g.y;
                    const double r = rsqrt(xr * xr + xi * xi);
                    st64[i] = make_double2(xr * r, xi * r);
                }
                __syncthreads();
                status = relax_phase<double, B>(J, st64, J.eps64, sw64, D, red);
            }
        } else {
            status = relax_phase<double, B>(J, st64, J.eps64, sw64, D, red);
        }

        if (J.state_out && local == 0) {
            // representative: theta_i - theta_{V-1} in (-pi, pi]
            const double2 gl = in64 ? st64[V - 1] : make_double2(st32[V - 1].x, st32[V - 1].y);
            for (int i = tid; i < V; i += B) {
                const double2 g = in64 ? st64[i] : make_double2(st32[i].x, st32[i].y);
                J.state_out[i] = rel_angle(g, gl);
            }
        }

        double F = 0.0, lam2 = NAN;
        uint64_t key_hi = 0, key_lo = 0;
        uint32_t paper_X = 0, flags = 0, lit = 0;
        if (status == GC_ST_CONVERGED && !(J.flags & GC_JOB_NO_TABLE)) {
            // ---- observables: u_l, a_l, w_l = Re u_l, F (eq. (3))
            double *sa = wscr;                   // [d][V] link angles
            double *sw = wscr + (uint64_t)d * V; // [d][V] link weights
            double facc = 0.0;
            for (int l = tid; l < d * V; l += B) {
                const int mu = l / V, i = l - mu * V;
                const int f = O.nbr[mu * V + i];
                const double2 u = O.U64[l];
                const double2 gi = st64[i], gf = st64[f];
                const double tr = u.x * gf.x - u.y * gf.y;
                const double ti = u.x * gf.y + u.y * gf.x;
                const double ur = gi.x * tr + gi.y * ti;
                const double ui = gi.x * ti - gi.y * tr;
                facc += 1.0 - ur;
                sa[l] = atan2(ui, ur);
                sw[l] = ur;
            }
            F = wg_sum<B>(facc, red);   // barrier inside also publishes sa/sw
            const double x = F / ((double)d * (double)V);
            paper_X = (uint32_t)(x * 1e8);

            // ---- integer key: plaquette wrap numbers, then line windings
            const uint64_t c0 = 0x243F6A8885A308D3ULL, c1 = 0x13198A2E03707344ULL;
            uint64_t h0 = 0, h1 = 0;
            int overflow = 0;
            for (int k = tid; k < O.n_elems; k += B) {
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
            h0 = wg_sum_u64<B>(h0, ured);
            h1 = wg_sum_u64<B>(h1, ured);
            const int ovf = wg_min_int<B>(overflow ? 0 : 1, ired);
            key_hi = mix64(h0 + (uint64_t)O.n_elems);
            key_lo = mix64(h1 + (uint64_t)O.n_elems);
            if (key_hi == 0) key_hi = 1;
            if (!ovf) flags |= GC_F_KEY_OVERFLOW;

            // ---- dedup
            if (tid == 0) {
                if (fixmode) {
                    flag_sh[0] = 1;
                } else {
                    bool claimed, is_min, failed;
                    table_insert(J, key_hi, key_lo, sid, F, claimed, is_min, failed);
                    flag_sh[0] = is_min ? 1 : 0;
                    if (claimed) atomicAdd(&J.cnt->distinct, 1ULL);
                    if (failed) atomicAdd(&J.cnt->errors, 1ULL);
                }
            }
            __syncthreads();
            const bool run_filter = flag_sh[0] != 0;
            __syncthreads();

            // ---- FP-operator filter for the lowest start of the key.  The
            // Lanczos vectors live in LDS: q_j in the single-precision state
            // region, q_{j-1} and the residual in the (no longer needed)
            // double-precision state region.
            if (run_filter) {
                const double sigma = 4.0 * d + 1.0;
                double *vq = lq;
                double *vp = reinterpret_cast<double *>(st64);
                double *vr = vp + V;
                // deterministic start vector orthogonal to the constant mode
                double acc = 0.0;
                for (int i = tid; i < V; i += B) {
                    const double r0 = (double)(mix64((uint64_t)i + 0x5851F42D4C957F2DULL) >> 11) * 0x1.0p-53 - 0.5;
                    vr[i] = r0;
                    vp[i] = 0.0;
                    acc += r0;
                }
                const double mean = wg_sum<B>(acc, red) / (double)V;
                acc = 0.0;
                for (int i = tid; i < V; i += B) {
                    const double r0 = vr[i] - mean;
                    vr[i] = r0;
                    acc += r0 * r0;
                }
                const double nrm = sqrt(wg_sum<B>(acc, red));
                for (int i = tid; i < V; i += B) vq[i] = vr[i] / nrm;
                __syncthreads();
                double beta_prev = 0.0, theta = INFINITY, theta_old = INFINITY;
                const int maxit = min(min(J.lanczos_max, GC_LMAX), V);
                int it = 0;
                bool conv = false;
                for (it = 0; it < maxit; ++it) {
                    double sq = 0.0, aq = 0.0;
                    for (int i = tid; i < V; i += B) sq += vq[i];
                    const double shift = sigma * wg_sum<B>(sq, red) / (double)V;
                    for (int i = tid; i < V; i += B) {
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
                    const double a_j = wg_sum<B>(aq, red);
                    acc = 0.0;
                    for (int i = tid; i < V; i += B) {
                        const double r = vr[i] - a_j * vq[i];
                        vr[i] = r;
                        acc += r * r;
                    }
                    const double b_j = sqrt(wg_sum<B>(acc, red));
                    if (tid == 0) {
                        alpha[it] = a_j;
                        beta[it] = b_j;
                    }
                    __syncthreads();
                    const bool breakdown = b_j <= 1e-13 * sigma;
                    if (((it + 1) % 8 == 0) || breakdown || it + 1 == maxit) {
                        theta = tridiag_min_eig<B>(alpha, beta, it + 1, ired);
                        if (breakdown || fabs(theta - theta_old) <= 1e-12 * fmax(1.0, fabs(theta))) {
                            conv = true;
                            ++it;
                            break;
                        }
                        theta_old = theta;
                    }
                    for (int i = tid; i < V; i += B) {
                        vp[i] = vq[i];
                        vq[i] = vr[i] / b_j;
                    }
                    beta_prev = b_j;
                    __syncthreads();
                }
                lam2 = theta;
                lit = (uint32_t)it;
                if (!conv) flags |= GC_F_LANCZOS_CAP;
                if (lam2 > J.lambda_tol) flags |= GC_F_IN_REGION;
                else if (lam2 < -J.lambda_tol) flags |= GC_F_SADDLE;
                else flags |= GC_F_SINGULAR;
                if (tid == 0) atomicAdd(&J.cnt->lanczos_runs, 1ULL);
            }
        }

        if (tid == 0 && fixmode) {
            J.fix[local].lambda2 = lam2;
            J.fix[local].flags = flags;
            J.fix[local].lanczos_iters = lit;
        } else if (tid == 0) {
            GcStartRec r;
            r.status = status;
            r.sweeps32 = (uint32_t)sw32;
            r.sweeps64 = (uint32_t)sw64;
            r.lanczos_iters = lit;
            r.F = F;
            r.D = D;
            r.lambda2 = lam2;
            r.key_hi = key_hi;
            r.key_lo = key_lo;
            r.paper_X = paper_X;
            r.flags = flags;
            J.rec[local] = r;
            atomicAdd(&J.cnt->starts_done, 1ULL);
            atomicAdd(status == GC_ST_CONVERGED ? &J.cnt->converged : &J.cnt->nonconverged, 1ULL);
            atomicAdd(&J.cnt->sweeps_total, (unsigned long long)(sw32 + sw64));
        }
        __syncthreads();
    }
}

__global__ void reset_kernel(GcJobDev J, unsigned long long *next)
{
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = gid; t <= J.table_mask; t += stride) {
        GcEntry e;
        e.key_hi = 0; e.key_lo = 0; e.hits = 0; e.first_start = ~0ULL;
        e.fmin_bits = ~0ULL; e.fmax_bits = 0; e.ready = 0; e.pad = 0; e.rep_start = ~0ULL;
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
        if (next) *next = 0ULL;
    }
}

// Find the table slot of a key (the table is complete when this runs).
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

// Representative of each copy: the lowest start id whose F lies within
// GC_F_SPREAD_PER_SITE (per site) of the lowest F reaching the key.  A start
// that stopped next to a saddle of the same class has a larger F and is not
// chosen.
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
        if (r.F - fmin <= tolF) atomicMin((unsigned long long *)&e->rep_start, (unsigned long long)(J.first_start + t));
    }
}

__global__ void finalize_kernel(GcJobDev J)
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

__global__ void zero_counter_kernel(unsigned long long *p) { *p = 0ULL; }

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

}  // namespace

size_t gc_solve_lds_bytes(int V, int /*precision*/)
{
    return 24 * (size_t)V + 2 * GC_LMAX * sizeof(double);
}

static hipError_t launch_solve_any(int block, const GcJobDev *jobs, int n_jobs, const uint64_t *prefix,
                                   unsigned long long *next, uint64_t total, const unsigned long long *total_dev,
                                   double *scratch, uint64_t scratch_stride, int grid, size_t lds_bytes, hipStream_t s)
{
    switch (block) {
    case 64:
        hipLaunchKernelGGL(solve_kernel<64>, dim3(grid), dim3(64), lds_bytes, s, jobs, n_jobs, prefix, next, total,
                           total_dev, scratch, scratch_stride);
        break;
    case 128:
        hipLaunchKernelGGL(solve_kernel<128>, dim3(grid), dim3(128), lds_bytes, s, jobs, n_jobs, prefix, next, total,
                           total_dev, scratch, scratch_stride);
        break;
    case 256:
        hipLaunchKernelGGL(solve_kernel<256>, dim3(grid), dim3(256), lds_bytes, s, jobs, n_jobs, prefix, next, total,
                           total_dev, scratch, scratch_stride);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t gc_solve_occupancy(int block, size_t lds_bytes, int *blocks_per_cu)
{
    switch (block) {
    case 64: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, solve_kernel<64>, 64, lds_bytes);
    case 128: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, solve_kernel<128>, 128, lds_bytes);
    case 256: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, solve_kernel<256>, 256, lds_bytes);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gc_launch_solve(int block, const GcJobDev *jobs, int n_jobs, const uint64_t *prefix,
                           unsigned long long *next, uint64_t total, double *scratch,
                           uint64_t scratch_stride, int grid, size_t lds_bytes, hipStream_t s)
{
    return launch_solve_any(block, jobs, n_jobs, prefix, next, total, nullptr, scratch, scratch_stride, grid,
                            lds_bytes, s);
}

hipError_t gc_launch_fixup(int block, const GcJobDev *fix_jobs_dev, const GcJobDev *jobs_host, int n_jobs,
                           unsigned long long *next, double *scratch, uint64_t scratch_stride, int grid,
                           size_t lds_bytes, hipStream_t s)
{
    for (int j = 0; j < n_jobs; ++j) {
        hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, next);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_solve_any(block, fix_jobs_dev + j, 1, nullptr, next, 0, jobs_host[j].n_fix, scratch,
                             scratch_stride, grid, lds_bytes, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(patch_kernel, dim3(64), dim3(256), 0, s, jobs_host[j]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gc_launch_reset(const GcJobDev *jobs_host, int n_jobs, unsigned long long *next, hipStream_t s)
{
    for (int j = 0; j < n_jobs; ++j) {
        const GcJobDev &J = jobs_host[j];
        uint64_t work = J.table_mask + 1 > J.n_starts ? J.table_mask + 1 : J.n_starts;
        int grid = (int)((work + 255) / 256);
        if (grid > 4096) grid = 4096;
        if (grid < 1) grid = 1;
        hipLaunchKernelGGL(reset_kernel, dim3(grid), dim3(256), 0, s, J, j == 0 ? next : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gc_launch_finalize(const GcJobDev *jobs_host, int n_jobs, hipStream_t s)
{
    for (int j = 0; j < n_jobs; ++j) {
        const GcJobDev &J = jobs_host[j];
        int rgrid = (int)((J.n_starts + 255) / 256);
        if (rgrid > 4096) rgrid = 4096;
        if (rgrid < 1) rgrid = 1;
        hipLaunchKernelGGL(rep_kernel, dim3(rgrid), dim3(256), 0, s, J);
        hipError_t e0 = hipGetLastError();
        if (e0 != hipSuccess) return e0;
        int grid = (int)((J.table_mask + 1 + 255) / 256);
        if (grid > 4096) grid = 4096;
        if (grid < 1) grid = 1;
        hipLaunchKernelGGL(finalize_kernel, dim3(grid), dim3(256), 0, s, J);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gc_launch_orbit_random(double *phi, int64_t n_links, uint64_t seed, uint64_t orbit_index, hipStream_t s)
{
    const int64_t blocks4 = (n_links + 3) / 4;
    const int grid = (int)((blocks4 + 255) / 256);
    hipLaunchKernelGGL(orbit_random_kernel, dim3(grid), dim3(256), 0, s, phi, n_links, seed, orbit_index);
    return hipGetLastError();
}
