// Wavefront-per-start solver for lattices with even extents (two colours).
//
// Each 64-lane wavefront relaxes one random start with its state resident in
// LDS and never synchronises with other wavefronts: a start finishes on its
// own schedule and the wavefront pulls the next start of its job from a
// per-job counter.  The workgroup only synchronises when it moves to another
// job (the orbit's coefficient table may be staged in LDS and is shared by
// its wavefronts).
//
// Layout (colour split, Sec. III checkerboard): site i has colour
// c = (sum_mu x_mu) mod 2 and half index h = i >> 1 (x_0 runs over an even
// extent, so sites 2h and 2h+1 have opposite colours).  A start's state is
// st[c][h] (complex), the update of (c, h) reads its 2d neighbours in
// st[1-c][.], and the orbit supplies per (c, h):
//   nb[c][h]      the 2d neighbour half indices (forward mu = 0..d-1, then backward)
//   coef[c][k][h] U_{i,k} for forward k, conj(U_{i-k,k}) for backward k,
// so that S_i = sum_k coef_k g_{n_k} (eqs. (4)-(5) in the eq. (3) convention).
//
// The stopping norm of sweep t needs div_i on the post-sweep state.  For the
// colour updated last it is formed right after the update; for colour 0 the
// staple S_i of the post-sweep state is exactly the one sweep t+1 computes
// first, so the norm of sweep t is completed there, before sweep t+1's new
// values are written, and the sweep is discarded if the norm has fallen
// below the threshold.  The arithmetic is that of a separate check pass.
#include "gc_common.h"
#include "gc_wave.h"

namespace {

using namespace gc;

// S for slot (c, h): sum_k coef[c][k][h] * st[1-c][nb_k]
template <int D, typename R>
__device__ __forceinline__ typename cx<R>::T staple(const typename cx<R>::T *__restrict__ coef,
                                                    const typename cx<R>::T *other, const uint4 nbp,
                                                    int c, int h, int half)
{
    using C = typename cx<R>::T;
    const uint32_t w[4] = {nbp.x, nbp.y, nbp.z, nbp.w};
    R ax = 0, ay = 0;
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        const int n = (int)((w[k >> 1] >> (16 * (k & 1))) & 0xFFFFu);
        const C u = coef[(c * 2 * D + k) * half + h];
        const C g = other[n];
        ax += u.x * g.x - u.y * g.y;
        ay += u.x * g.y + u.y * g.x;
    }
    C s;
    s.x = ax;
    s.y = ay;
    return s;
}

// New value of g at one site from its staple (relaxation or over-relaxation).
template <typename R>
__device__ __forceinline__ typename cx<R>::T local_update(typename cx<R>::T g0, typename cx<R>::T s, R omega, bool relax)
{
    using C = typename cx<R>::T;
    const R n2 = s.x * s.x + s.y * s.y;
    if (n2 == (R)0) return g0;
    const R r = rsq(n2);
    const R hx = s.x * r, hy = s.y * r;
    C g;
    if (relax) {
        g.x = hx;
        g.y = hy;
    } else {
        const R zx = g0.x * hx + g0.y * hy;
        const R zy = g0.x * hy - g0.y * hx;
        R wx = (R)1 + omega * (zx - (R)1);
        R wy = omega * zy;
        const R rw = rsq(wx * wx + wy * wy);
        wx *= rw;
        wy *= rw;
        g.x = g0.x * wx - g0.y * wy;
        g.y = g0.x * wy + g0.y * wx;
    }
    return g;
}

// Sweeps of one precision on the wave's state st[2][half].  Returns status.
template <int D, typename R, int NS>
__device__ int relax_wave(const GcJobDev &J, const GcWaveOrbit &WO, const typename cx<R>::T *__restrict__ coef,
                          typename cx<R>::T *st, double eps, uint64_t &sweeps, double &D_out)
{
    using C = typename cx<R>::T;
    const int lane = threadIdx.x & 63;
    const int half = WO.half;
    C *st0 = st, *st1 = st + half;
    const R omega = (R)J.omega;
    const bool relax = (omega == (R)1);
    const uint64_t check = J.check_every > 0 ? (uint64_t)J.check_every : 1;
    const bool maxabs = J.stop_norm != 0;
    const uint4 *__restrict__ nb0 = WO.nb;
    const uint4 *__restrict__ nb1 = WO.nb + half;

    uint64_t t = 0;
    double acc1 = 0.0;           // colour-1 part of the norm of sweep t
    int status = GC_ST_NONCONVERGED;
    D_out = INFINITY;
    // sweep t + 1 reads the colour-0 staples of the state after sweep t;
    // when t is a check point they complete the norm of sweep t.
    for (;;) {
        const bool pending = (t > 0) && (t % check == 0 || t == J.max_sweeps);
        const bool last = (t == J.max_sweeps);
        const int z = opaque_zero();
        // ---- colour 0 (and the colour-0 part of the pending norm)
        C gnew[NS];
        double acc0 = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int h = lane + 64 * k;
            if (h < half) {
                const C s = staple<D, R>(coef, st1, nb0[h + z], 0, h + z, half);
                const C g0 = st0[h];
                if (pending) {
                    const double dv = (double)(g0.x * s.y - g0.y * s.x);
                    acc0 = maxabs ? fmax(acc0, fabs(dv)) : acc0 + dv * dv;
                }
                gnew[k] = last ? g0 : local_update<R>(g0, s, omega, relax);
            }
        }
        if (pending) {
            const double Dn = maxabs ? fmax(wave_max(acc0), acc1) : (wave_sum(acc0) + acc1) / (double)(2 * half);
            D_out = Dn;
            if (!(Dn == Dn)) { status = GC_ST_BADNUM; break; }
            if (Dn < eps) { status = GC_ST_CONVERGED; break; }
        }
        if (last) break;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int h = lane + 64 * k;
            if (h < half) st0[h] = gnew[k];
        }
        wave_sync();
        // ---- colour 1, with its part of the norm of this sweep
        ++t;
        const bool chk = (t % check == 0 || t == J.max_sweeps);
        double a1 = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int h = lane + 64 * k;
            if (h < half) {
                const C s = staple<D, R>(coef, st0, nb1[h + z], 1, h + z, half);
                const C g = local_update<R>(st1[h], s, omega, relax);
                st1[h] = g;
                if (chk) {
                    const double dv = (double)(g.x * s.y - g.y * s.x);
                    a1 = maxabs ? fmax(a1, fabs(dv)) : a1 + dv * dv;
                }
            }
        }
        if (chk) acc1 = maxabs ? wave_max(a1) : wave_sum(a1);
        wave_sync();
    }
    sweeps = t;
    return status;
}

template <int D, int NS>
__device__ void relax_start_wave(const GcJobDev &J, const GcWaveOrbit &WO, const double2 *coef64,
                                 const float2 *coef32, double2 *st64, float2 *st32, float2 *bounce, uint64_t local)
{
    const int lane = threadIdx.x & 63;
    const GcOrbitDev &O = J.orb;
    const int V = O.V;
    const uint64_t sid = J.first_start + local;

    // random start, written at its colour-split position loc[i]
    for (int b = lane; 4 * b < V; b += 64) {
        uint64_t c[4];
        start_block(J.start_seed, sid, O.orbit_index, (uint64_t)b, c);
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            const int i = 4 * b + k;
            if (i < V) {
                double sn, cs;
                sincos(angle_of(c[k]), &sn, &cs);
                const int p = WO.loc[i];
                if (J.precision == 1) st32[p] = make_float2((float)cs, (float)sn);
                else st64[p] = make_double2(cs, sn);
            }
        }
    }
    wave_sync();

    uint64_t sw32 = 0, sw64 = 0;
    double Dn = INFINITY;
    int status;
    bool in64 = J.precision != 1;
    if (J.precision == 1) {
        status = relax_wave<D, float, NS>(J, WO, coef32, st32, J.eps32, sw32, Dn);
        if (status == GC_ST_CONVERGED) {
            // promotion g64 = normalise((double) g32): both states share the
            // wave's LDS region, so each lane bounces its entries through
            // its private scratch
            in64 = true;
            for (int p = lane; p < V; p += 64) bounce[p] = st32[p];
            wave_sync();
            for (int p = lane; p < V; p += 64) {
                const float2 g = bounce[p];
                const double xr = (double)g.x, xi = (double)g.y;
                const double r = rsqrt(xr * xr + xi * xi);
                st64[p] = make_double2(xr * r, xi * r);
            }
            wave_sync();
            status = relax_wave<D, double, NS>(J, WO, coef64, st64, J.eps64, sw64, Dn);
        }
    } else {
        status = relax_wave<D, double, NS>(J, WO, coef64, st64, J.eps64, sw64, Dn);
    }
    // final state in natural site order
    double2 *out = J.states + local * (uint64_t)V;
    for (int i = lane; i < V; i += 64) {
        const int p = WO.loc[i];
        out[i] = in64 ? st64[p] : make_double2((double)st32[p].x, (double)st32[p].y);
    }
    if (lane == 0) record_relax(J, local, status, sw32, sw64, Dn);
    wave_sync();
}

// WG = WAVES wavefronts.  LDS: [coef64 | coef32 staged when coef_lds] then
// per wave a 16V-byte state region (double2[V], or float2[V] in the single-
// precision phase).
template <int D, int NS, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void wave_kernel(const GcJobDev *__restrict__ jobs,
                                                          const GcWaveOrbit *__restrict__ worbs, int n_jobs,
                                                          unsigned long long *job_next, int coef_lds,
                                                          float2 *bounce_all)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cur_job;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    int j0 = (int)(blockIdx.x % (unsigned)n_jobs);
    for (int round = 0; round < n_jobs; ++round) {
        if (threadIdx.x == 0) {
            int pick = -1;
            for (int k = 0; k < n_jobs; ++k) {
                const int j = (j0 + k) % n_jobs;
                if (__hip_atomic_load(&job_next[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < jobs[j].n_starts) {
                    pick = j;
                    break;
                }
            }
            cur_job = pick;
        }
        __syncthreads();
        const int jn = cur_job;
        __syncthreads();
        if (jn < 0) break;
        const GcJobDev &J = jobs[jn];
        const GcWaveOrbit &WO = worbs[jn];
        const int V = J.orb.V;
        const int ncoef = 2 * D * V;      // complex entries per precision
        const double2 *coef64 = WO.coef64;
        const float2 *coef32 = WO.coef32;
        size_t off = 0;
        if (coef_lds) {
            double2 *c64 = reinterpret_cast<double2 *>(smem);
            for (int t = threadIdx.x; t < ncoef; t += 64 * WAVES) c64[t] = WO.coef64[t];
            coef64 = c64;
            off = 16 * (size_t)ncoef;
            if (J.precision == 1) {
                float2 *c32 = reinterpret_cast<float2 *>(smem + off);
                for (int t = threadIdx.x; t < ncoef; t += 64 * WAVES) c32[t] = WO.coef32[t];
                coef32 = c32;
                off += 8 * (size_t)ncoef;
            }
        }
        __syncthreads();
        double2 *st64 = reinterpret_cast<double2 *>(smem + off + (size_t)wave * 16 * V);
        float2 *st32 = reinterpret_cast<float2 *>(st64);
        for (;;) {
            unsigned long long s = 0;
            if (lane == 0) s = atomicAdd(&job_next[jn], 1ULL);
            s = __shfl(s, 0, 64);
            if (s >= J.n_starts) break;
            float2 *bounce = bounce_all + ((uint64_t)blockIdx.x * WAVES + wave) * (uint64_t)V;
            relax_start_wave<D, NS>(J, WO, coef64, coef32, st64, st32, bounce, s);
        }
        __syncthreads();
        j0 = jn;
    }
}

template <int D, int NS, int WAVES>
hipError_t launch_t(const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs, unsigned long long *job_next,
                    int coef_lds, float2 *bounce, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((wave_kernel<D, NS, WAVES>), dim3(grid), dim3(64 * WAVES), lds, s, jobs, worbs, n_jobs,
                       job_next, coef_lds, bounce);
    return hipGetLastError();
}

template <int D, int NS, int WAVES>
hipError_t occ_t(size_t lds, int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, wave_kernel<D, NS, WAVES>, 64 * WAVES, lds);
}

}  // namespace

// NS = slots per lane per colour = ceil(half / 64); instantiated for the
// half-volumes up to 2048 sites (V <= 4096).
#define GC_WAVE_DISPATCH(FN, ...)                                                              \
    switch (d) {                                                                               \
    case 1: return ns <= 1 ? FN<1, 1, 4>(__VA_ARGS__) : ns <= 4 ? FN<1, 4, 4>(__VA_ARGS__)     \
                 : ns <= 12 ? FN<1, 12, 4>(__VA_ARGS__) : FN<1, 32, 4>(__VA_ARGS__);           \
    case 2: return ns <= 1 ? FN<2, 1, 4>(__VA_ARGS__) : ns <= 2 ? FN<2, 2, 4>(__VA_ARGS__)     \
                 : ns <= 4 ? FN<2, 4, 4>(__VA_ARGS__) : ns <= 12 ? FN<2, 12, 4>(__VA_ARGS__)   \
                 : FN<2, 32, 4>(__VA_ARGS__);                                                  \
    case 3: return ns <= 2 ? FN<3, 2, 4>(__VA_ARGS__) : ns <= 4 ? FN<3, 4, 4>(__VA_ARGS__)     \
                 : ns <= 8 ? FN<3, 8, 4>(__VA_ARGS__) : FN<3, 32, 4>(__VA_ARGS__);             \
    case 4: return ns <= 1 ? FN<4, 1, 4>(__VA_ARGS__) : ns <= 2 ? FN<4, 2, 4>(__VA_ARGS__)     \
                 : ns <= 4 ? FN<4, 4, 4>(__VA_ARGS__) : ns <= 11 ? FN<4, 11, 4>(__VA_ARGS__)   \
                 : FN<4, 32, 4>(__VA_ARGS__);                                                  \
    default: return hipErrorInvalidValue;                                                      \
    }

hipError_t gc_wave_occupancy(int d, int ns, size_t lds, int *per_cu)
{
    GC_WAVE_DISPATCH(occ_t, lds, per_cu)
}

hipError_t gc_launch_wave(int d, int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,
                          unsigned long long *job_next, int coef_lds, float2 *bounce, int grid, size_t lds,
                          hipStream_t s)
{
    GC_WAVE_DISPATCH(launch_t, jobs, worbs, n_jobs, job_next, coef_lds, bounce, grid, lds, s)
}

