// Maximal Abelian reduction of an SU(2) configuration (Sec. I): the Landau
// functional of eq. (1) is stated for SU(N_c), and the Neuberger problem of
// SU(N_c) lies in its maximal Abelian subgroup U(1)^{N_c - 1}, the coset part
// being free of it.  The configuration is gauge-fixed on the coset SU(2)/U(1)
// to the maximal Abelian gauge -- R = sum_{x,mu} 1/2 Tr(s3 U' s3 U'^dagger),
// U' = g_x U_{x,mu} g_{x+mu}^dagger, maximised site by site, colour by
// colour -- and the diagonal phases of U' are the compact U(1) orbit whose
// Landau-gauge copies the rest of the library enumerates.
//
// Quaternions q = (q0, q1, q2, q3) stand for q0 + i (q1 s1 + q2 s2 + q3 s3).
// The arithmetic is written out in the order of the definitions, without
// floating-point contraction, so that a sweep rounds like the plain
// double-precision sequence of operations it states.
#include "gc_common.h"
#include "gc_internal.h"

#pragma clang fp contract(off)

namespace {

using namespace gc;

struct Quat {
    double w, x, y, z;   // q0, q1, q2, q3
};

// (i s_a)(i s_b) = -delta_ab - i eps_abc s_c
__device__ __forceinline__ Quat qmul(const Quat &p, const Quat &q)
{
    Quat r;
    r.w = p.w * q.w - p.x * q.x - p.y * q.y - p.z * q.z;
    r.x = p.w * q.x + q.w * p.x - (p.y * q.z - p.z * q.y);
    r.y = p.w * q.y + q.w * p.y - (p.z * q.x - p.x * q.z);
    r.z = p.w * q.z + q.w * p.z - (p.x * q.y - p.y * q.x);
    return r;
}

__device__ __forceinline__ Quat qconj(const Quat &q) { return Quat{q.w, -q.x, -q.y, -q.z}; }

// b with Q s3 Q^dagger = b . s: b3 = |alpha|^2 - |beta|^2, b1 - i b2 =
// -2 alpha beta for Q = [[alpha, beta], [-conj(beta), conj(alpha)]],
// alpha = q0 + i q3, beta = q2 + i q1
__device__ __forceinline__ void rot3(const Quat &q, double &b1, double &b2, double &b3)
{
    b1 = -2.0 * (q.w * q.y - q.x * q.z);
    b2 = 2.0 * (q.w * q.x + q.y * q.z);
    b3 = q.w * q.w + q.z * q.z - q.x * q.x - q.y * q.y;
}

// The g with g^dagger s3 g = n . s whose conjugate h = g^dagger has a real,
// non-negative diagonal element: alpha = sqrt((1 + n3)/2), beta =
// -(n1 - i n2)/(2 alpha) (alpha = 0, beta = 1 at n3 = -1)
__device__ __forceinline__ Quat from_axis3(double n1, double n2, double n3)
{
    const double a = sqrt(0.5 * (1.0 + n3));
    double br = 1.0, bi = 0.0;
    if (a > 0.0) {
        const double den = 2.0 * a;
        br = -n1 / den;
        bi = n2 / den;
    }
    return Quat{a, -bi, -br, -0.0};
}

__device__ __forceinline__ Quat load_q(const double *__restrict__ p, size_t k)
{
    const double4 v = reinterpret_cast<const double4 *>(p)[k];
    return Quat{v.x, v.y, v.z, v.w};
}

constexpr int kMagBlock = 1024;

// Sum over the workgroup in a fixed order (wavefront sums, then the waves in
// order); every thread returns the total.
__device__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kMagBlock / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// One workgroup per configuration: g (V quaternions) in LDS, the links in
// global memory.  links [d][V] quaternions, nbr [2d][V] (forward, then
// backward), csite [V]: the sites of colour 0, then those of colour 1 (V/2
// each).  A sweep updates colour 0, then colour 1: at site x, R depends on
// g_x only through n . M with n . s = g_x^dagger s3 g_x and M = sum_mu
// [w_mu + y_mu] (mu ascending, forward then backward), W = U_{x,mu}
// g_{x+mu}^dagger with w . s = W s3 W^dagger and Y = g_{x-mu} U_{x-mu,mu}
// with y . s = Y^dagger s3 Y, so n = M/|M| (M = 0 leaves g_x unchanged).
// D = (1/V) sum_x |n_x - n_x^old|^2 over a sweep; the reduction stops after
// the first sweep with D < eps, or after max_sweeps.  Then phi[mu][x] = arg
// of the diagonal element of U'_{x,mu} and out the sweeps, R/(dV) and
// whether D fell below eps.
__global__ __launch_bounds__(kMagBlock) void mag_kernel(const double *__restrict__ links, const int *__restrict__ nbr,
                                                        const int *__restrict__ csite, int d, int V, double eps,
                                                        uint64_t max_sweeps, double *__restrict__ phi,
                                                        GcMagOut *__restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kMagBlock / 64];
    Quat *g = reinterpret_cast<Quat *>(smem);
    const int tid = (int)threadIdx.x;
    const int half = V / 2;
    for (int x = tid; x < V; x += kMagBlock) g[x] = Quat{1.0, 0.0, 0.0, 0.0};
    __syncthreads();
    uint64_t sweeps = 0;
    int converged = 0;
    while (sweeps < max_sweeps) {
        double acc = 0.0;
        for (int c = 0; c < 2; ++c) {
            for (int j = tid; j < half; j += kMagBlock) {
                const int x = csite[c * half + j];
                double m1 = 0.0, m2 = 0.0, m3 = 0.0;
                for (int mu = 0; mu < d; ++mu) {
                    const int f = nbr[mu * V + x], b = nbr[(d + mu) * V + x];
                    double b1, b2, b3;
                    const Quat W = qmul(load_q(links, (size_t)mu * V + x), qconj(g[f]));
                    rot3(W, b1, b2, b3);
                    m1 = m1 + b1;
                    m2 = m2 + b2;
                    m3 = m3 + b3;
                    const Quat Y = qmul(g[b], load_q(links, (size_t)mu * V + b));
                    rot3(qconj(Y), b1, b2, b3);
                    m1 = m1 + b1;
                    m2 = m2 + b2;
                    m3 = m3 + b3;
                }
                const double mm = m1 * m1 + m2 * m2 + m3 * m3;
                if (mm > 0.0) {
                    double o1, o2, o3;
                    rot3(qconj(g[x]), o1, o2, o3);
                    const double s = sqrt(mm);
                    const double n1 = m1 / s, n2 = m2 / s, n3 = m3 / s;
                    g[x] = from_axis3(n1, n2, n3);
                    const double e1 = n1 - o1, e2 = n2 - o2, e3 = n3 - o3;
                    acc += e1 * e1 + e2 * e2 + e3 * e3;
                }
            }
            __syncthreads();
        }
        ++sweeps;
        const double D = block_sum(acc, red) / (double)V;
        if (D < eps) {
            converged = 1;
            break;
        }
    }
    double racc = 0.0;
    for (int l = tid; l < d * V; l += kMagBlock) {
        const int mu = l / V, x = l - mu * V;
        const Quat Up = qmul(qmul(g[x], load_q(links, (size_t)l)), qconj(g[nbr[mu * V + x]]));
        double b1, b2, b3;
        rot3(Up, b1, b2, b3);
        racc += b3;
        phi[l] = atan2(Up.z, Up.w);
    }
    const double R = block_sum(racc, red) / (double)(d * V);
    if (tid == 0) {
        out->sweeps = sweeps;
        out->R = R;
        out->converged = converged;
    }
}

}  // namespace

size_t gc_mag_lds_bytes(int V) { return sizeof(Quat) * (size_t)V; }

hipError_t gc_launch_mag(const double *links, const int *nbr, const int *csite, int d, int V, double eps,
                         uint64_t max_sweeps, double *phi, GcMagOut *out, hipStream_t s)
{
    hipLaunchKernelGGL(mag_kernel, dim3(1), dim3(kMagBlock), gc_mag_lds_bytes(V), s, links, nbr, csite, d, V, eps,
                       max_sweeps, phi, out);
    return hipGetLastError();
}
