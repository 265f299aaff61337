// Relaxation kernel for any lattice (any number of checkerboard colours):
// one workgroup holds one random start in LDS, in natural site order, and
// pulls the next start from a device-wide counter when its start is done.
//
// Per start: Philox start angles (Sec. III) -> g; colour c = 0..K-1, every
// site of colour c updated concurrently (Sec. III) by the local maximisation
// of eqs. (4)-(5) in the eq. (3) convention; after every check point the
// stopping norm (1/V) sum div_i^2 (or max |div_i|, the paper's rule),
// div_i = Im(conj(g_i) S_i), on the post-sweep state; FP32 phase then FP64
// polish in mixed mode.  The final double-precision state goes to HBM for the
// post kernel.
#include "gc_common.h"

namespace {

using namespace gc;

template <int B>
__device__ __forceinline__ double wg_sum(double v, double *red)
{
    v = wave_sum(v);
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
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int k = 1; k < B / 64; ++k) s = fmax(s, red[k]);
    return s;
}

template <typename R> __device__ __forceinline__ const typename cx<R>::T *links(const GcOrbitDev &O);
template <> __device__ __forceinline__ const flt2 *links<float>(const GcOrbitDev &O)
{
    return reinterpret_cast<const flt2 *>(O.U32);
}
template <> __device__ __forceinline__ const dbl2 *links<double>(const GcOrbitDev &O)
{
    return reinterpret_cast<const dbl2 *>(O.U64);
}

// S_i = sum_mu [U_{i,mu} g_{i+mu} + conj(U_{i-mu,mu}) g_{i-mu}], mu ascending
template <typename R>
__device__ __forceinline__ typename cx<R>::T staple(const GcOrbitDev &O, const typename cx<R>::T *__restrict__ U,
                                                    const typename cx<R>::T *st, int i)
{
    using C = typename cx<R>::T;
    const int V = O.V, d = O.d;
    R ax = 0, ay = 0;
    for (int mu = 0; mu < d; ++mu) {
        const int f = O.nbr[mu * V + i];
        const int b = O.nbr[(d + mu) * V + i];
        const C u = U[mu * V + i];
        const C gf = st[f];
        ax += u.x * gf.x - u.y * gf.y;
        ay += u.x * gf.y + u.y * gf.x;
        const C v = U[mu * V + b];
        const C gb = st[b];
        ax += v.x * gb.x + v.y * gb.y;
        ay += v.x * gb.y - v.y * gb.x;
    }
    C s;
    s.x = ax;
    s.y = ay;
    return s;
}

// Sweeps of one precision until the stopping norm is below eps (checked
// every check_every sweeps and at the cap), or, with fixed, exactly cap
// sweeps with the norm taken after the last (batch-synchronous pass).
template <typename R, int B>
__device__ int relax_phase(const GcJobDev &J, typename cx<R>::T *st, double eps, uint64_t cap, bool fixed,
                           uint64_t &sweeps, double &D, double *red)
{
    using C = typename cx<R>::T;
    const GcOrbitDev &O = J.orb;
    const C *__restrict__ U = links<R>(O);
    const int V = O.V, K = O.K, tid = threadIdx.x;
    const R omega = (R)J.omega;
    const bool relax = (omega == (R)1);
    const uint64_t check = J.check_every > 0 ? (uint64_t)J.check_every : 1;
    uint64_t t = 0;
    int status = GC_ST_NONCONVERGED;
    D = INFINITY;
    while (t < cap) {
        for (int c = 0; c < K; ++c) {
            const int lo = O.coff[c], hi = O.coff[c + 1];
            for (int p = lo + tid; p < hi; p += B) {
                const int i = O.perm[p];
                const C sv = staple<R>(O, U, st, i);
                st[i] = relax ? local_update<true, R>(st[i], sv, omega) : local_update<false, R>(st[i], sv, omega);
            }
            __syncthreads();
        }
        ++t;
        if ((!fixed && t % check == 0) || t == cap) {
            double acc = 0.0;
            for (int i = tid; i < V; i += B) {
                const C s = staple<R>(O, U, st, i);
                const C g = st[i];
                const double dv = (double)(g.x * s.y - g.y * s.x);
                acc = J.stop_norm ? fmax(acc, fabs(dv)) : acc + dv * dv;
            }
            D = J.stop_norm ? wg_max<B>(acc, red) : wg_sum<B>(acc, red) / (double)V;
            if (!(D == D)) { status = GC_ST_BADNUM; break; }
            if (D < eps) {
                status = GC_ST_CONVERGED;
                if (!fixed) break;
            } else {
                status = GC_ST_NONCONVERGED;
            }
        }
    }
    sweeps = t;
    return status;
}

template <int B>
__global__ __launch_bounds__(B) void relax_wg_kernel(const GcJobDev *__restrict__ jobs, int n_jobs,
                                                     const uint64_t *__restrict__ prefix, unsigned long long *next,
                                                     uint64_t total)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[B / 64];
    __shared__ unsigned long long claim;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) claim = atomicAdd(next, 1ULL);
        __syncthreads();
        const uint64_t s = uniform((uint64_t)claim);
        __syncthreads();
        if (s >= total) break;
        int jn = 0;
        while (jn + 1 < n_jobs && prefix[jn + 1] <= s) ++jn;
        jn = uniform(jn);
        const GcJobDev &J = jobs[jn];
        const GcOrbitDev &O = J.orb;
        const int V = O.V;
        const uint64_t local = s - prefix[jn];
        const uint64_t sid = J.first_start + local;
        dbl2 *st64 = reinterpret_cast<dbl2 *>(smem);
        flt2 *st32 = reinterpret_cast<flt2 *>(smem + 16 * (size_t)V);

        for (int b = tid; 4 * b < V; b += B) {
            uint64_t c[4];
            // the caller's start angles, else Philox (the block is skipped then)
            if (!J.theta_init) start_block(J.start_seed, sid, O.orbit_index, (uint64_t)b, c);
#pragma unroll 1
            for (int k = 0; k < 4; ++k) {
                const int i = 4 * b + k;
                if (i < V) {
                    double sn, cs;
                    sincos(J.theta_init ? J.theta_init[local * (uint64_t)V + i] : angle_of(c[k]), &sn, &cs);
                    if (J.precision == 1) st32[i] = flt2{(float)cs, (float)sn};
                    else st64[i] = dbl2{cs, sn};
                }
            }
        }
        __syncthreads();

        uint64_t sw32 = 0, sw64 = 0;
        double D = INFINITY;
        int status;
        bool in64 = J.precision != 1;
        const bool fixed = (J.flags & GC_JOB_SYNC2) != 0;
        const uint64_t cap = fixed ? (uint64_t)J.fixed_sweeps[local] : J.max_sweeps;
        if (J.precision == 1) {
            status = relax_phase<float, B>(J, st32, J.eps32, J.max_sweeps, false, sw32, D, red);
            if (status == GC_ST_CONVERGED) {
                in64 = true;
                for (int i = tid; i < V; i += B) {
                    const flt2 g = st32[i];
                    const double xr = (double)g.x, xi = (double)g.y;
                    const double r = rsqrt(xr * xr + xi * xi);
                    st64[i] = dbl2{xr * r, xi * r};
                }
                __syncthreads();
                status = relax_phase<double, B>(J, st64, J.eps64, J.max_sweeps, false, sw64, D, red);
            }
        } else {
            status = relax_phase<double, B>(J, st64, J.eps64, cap, fixed, sw64, D, red);
        }
        dbl2 *out = reinterpret_cast<dbl2 *>(J.states + local * (uint64_t)V);
        for (int i = tid; i < V; i += B)
            out[i] = in64 ? st64[i] : dbl2{(double)st32[i].x, (double)st32[i].y};
        if (tid == 0) record_relax(J, local, status, sw32, sw64, D);
        __syncthreads();
    }
}

}  // namespace

size_t gc_relax_wg_lds_bytes(int V) { return 24 * (size_t)V; }

hipError_t gc_relax_wg_occupancy(int block, size_t lds_bytes, int *blocks_per_cu)
{
    switch (block) {
    case 64: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, relax_wg_kernel<64>, 64, lds_bytes);
    case 128: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, relax_wg_kernel<128>, 128, lds_bytes);
    case 256: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, relax_wg_kernel<256>, 256, lds_bytes);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gc_launch_relax_wg(int block, const GcJobDev *jobs, int n_jobs, const uint64_t *prefix,
                              unsigned long long *next, uint64_t total, int grid, size_t lds_bytes, hipStream_t s)
{
    switch (block) {
    case 64:
        hipLaunchKernelGGL(relax_wg_kernel<64>, dim3(grid), dim3(64), lds_bytes, s, jobs, n_jobs, prefix, next, total);
        break;
    case 128:
        hipLaunchKernelGGL(relax_wg_kernel<128>, dim3(grid), dim3(128), lds_bytes, s, jobs, n_jobs, prefix, next, total);
        break;
    case 256:
        hipLaunchKernelGGL(relax_wg_kernel<256>, dim3(grid), dim3(256), lds_bytes, s, jobs, n_jobs, prefix, next, total);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
