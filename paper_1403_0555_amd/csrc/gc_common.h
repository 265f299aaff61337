// Device helpers shared by the enumerator's kernels.
#pragma once

#include "gc_internal.h"

#include <math.h>

namespace gc {

constexpr double kPi = 3.14159265358979311599796346854;
constexpr double kTwoPi = 6.28318530717958623199592693709;

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64 -> 128-bit products, key bumped by the Weyl constants each round.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// Uniform angle in [-pi, pi): fl(fl(u 2pi) - pi), u = (r >> 11) 2^-53, with
// contraction off so that the product is rounded before the subtraction.
__device__ __forceinline__ double angle_of(uint64_t r)
{
#pragma clang fp contract(off)
    const double u = (double)(r >> 11) * 0x1.0p-53;
    const double t = u * kTwoPi;
    return t - kPi;
}

// SplitMix64 output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Random start angle of site i of start sid (Philox block i/4, word i%4).
__device__ __forceinline__ void start_block(uint64_t start_seed, uint64_t sid, uint64_t orbit_index, uint64_t b,
                                            uint64_t out[4])
{
    out[0] = b;
    out[1] = sid;
    out[2] = orbit_index;
    out[3] = 0x53ULL;
    philox4x64_10(out, start_seed, 1ULL);
}

// Wavefront-level ordering of LDS traffic: every lane's earlier LDS writes
// are visible to every lane's later reads (LDS instructions of one wave
// execute in order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane ordering of global-memory traffic inside one wavefront.
__device__ __forceinline__ void wave_sync_global()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Reductions over the 64 lanes of a wavefront; every lane ends with the same
// value and the association order is fixed.  Within each row of 16 lanes
// the values are combined through DPP lane permutations (quad swaps, then
// the half-row and row mirrors); the four row results are then combined as
// (r0 + r1) + (r2 + r3) through the cross-row swaps of gfx950
// (v_permlane16_swap, v_permlane32_swap), so nothing touches LDS or scalar
// registers until the wave-uniform result is read from the first lane.
template <int CTRL> __device__ __forceinline__ int dpp32(int v)
{
    // every row and bank enabled: no lane keeps an old value, so none is
    // initialised
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ double dpp64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp32<CTRL>((int)b), hi = dpp32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double first_lane(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int kDppQuadSwap1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadSwap2 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppRowMirror = 0x140;  // row_mirror

// Cross-row pairs.  With both operands holding v, permlane16_swap leaves in
// every lane the value of its even row (first result) and of its odd row
// (second result) of the same row pair; permlane32_swap does the same for
// the lower and upper half-waves.  The two halves of a double take the same
// swap.
struct RowPair {
    double lo, hi;   // the even (lower) and the odd (upper) member of the pair
};
template <int W> __device__ __forceinline__ RowPair row_pair(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned l = (unsigned)b, h = (unsigned)(b >> 32);
    const auto sl = W == 16 ? __builtin_amdgcn_permlane16_swap(l, l, false, false)
                            : __builtin_amdgcn_permlane32_swap(l, l, false, false);
    const auto sh = W == 16 ? __builtin_amdgcn_permlane16_swap(h, h, false, false)
                            : __builtin_amdgcn_permlane32_swap(h, h, false, false);
    return {__longlong_as_double(((long long)sh[0] << 32) | (long long)sl[0]),
            __longlong_as_double(((long long)sh[1] << 32) | (long long)sl[1])};
}
template <int W> __device__ __forceinline__ int row_pair_min(int v)
{
    const auto s = W == 16 ? __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false)
                           : __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    return min((int)s[0], (int)s[1]);
}

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp64<kDppQuadSwap1>(v);
    v += dpp64<kDppQuadSwap2>(v);
    v += dpp64<kDppHalfMirror>(v);
    v += dpp64<kDppRowMirror>(v);
    RowPair p = row_pair<16>(v);
    v = p.lo + p.hi;
    p = row_pair<32>(v);
    return first_lane(p.lo + p.hi);
}
// N sums at once, step by step across the values: the lane moves of one
// value fill the waits the others' additions need.  Same association order
// as wave_sum for each value; the results stay in vector registers (equal
// in every lane).
template <int N> __device__ __forceinline__ void wave_sum_n(double (&v)[N])
{
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] += dpp64<kDppQuadSwap1>(v[n]);
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] += dpp64<kDppQuadSwap2>(v[n]);
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] += dpp64<kDppHalfMirror>(v[n]);
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] += dpp64<kDppRowMirror>(v[n]);
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const RowPair p = row_pair<16>(v[n]);
        v[n] = p.lo + p.hi;
    }
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const RowPair p = row_pair<32>(v[n]);
        v[n] = p.lo + p.hi;
    }
}
__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp64<kDppQuadSwap1>(v));
    v = fmax(v, dpp64<kDppQuadSwap2>(v));
    v = fmax(v, dpp64<kDppHalfMirror>(v));
    v = fmax(v, dpp64<kDppRowMirror>(v));
    RowPair p = row_pair<16>(v);
    v = fmax(p.lo, p.hi);
    p = row_pair<32>(v);
    return first_lane(fmax(p.lo, p.hi));
}
__device__ __forceinline__ double wave_min(double v)
{
    v = fmin(v, dpp64<kDppQuadSwap1>(v));
    v = fmin(v, dpp64<kDppQuadSwap2>(v));
    v = fmin(v, dpp64<kDppHalfMirror>(v));
    v = fmin(v, dpp64<kDppRowMirror>(v));
    RowPair p = row_pair<16>(v);
    v = fmin(p.lo, p.hi);
    p = row_pair<32>(v);
    return first_lane(fmin(p.lo, p.hi));
}
__device__ __forceinline__ int wave_min_int(int v)
{
    v = min(v, dpp32<kDppQuadSwap1>(v));
    v = min(v, dpp32<kDppQuadSwap2>(v));
    v = min(v, dpp32<kDppHalfMirror>(v));
    v = min(v, dpp32<kDppRowMirror>(v));
    v = row_pair_min<16>(v);
    v = row_pair_min<32>(v);
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Values known to be equal on every lane (broadcast through LDS or a
// shuffle): reading lane 0 puts them in scalar registers, so that whatever is
// indexed by them (job descriptors, start records) is loaded once per wave.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// A zero the optimiser cannot see through.  Indexing per-site tables with it
// inside a loop keeps them from being hoisted into registers.
__device__ __forceinline__ int opaque_zero()
{
    int z = 0;
    asm volatile("" : "+v"(z));
    return z;
}

// Address-space views: LDS (3) and global (1) pointers make the compiler emit
// ds_* or global_* instructions instead of generic flat accesses.
template <typename T> using lds_ptr = __attribute__((address_space(3))) T *;
template <typename T> using glb_ptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ glb_ptr<T> as_global(T *p) { return (glb_ptr<T>)p; }
template <typename T> __device__ __forceinline__ lds_ptr<T> as_lds(T *p) { return (lds_ptr<T>)p; }

// Complex numbers as clang vector types: builtin, so they load and store
// through any address space.
typedef float flt2 __attribute__((ext_vector_type(2)));
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename R> struct cx;
template <> struct cx<float> { using T = flt2; };
template <> struct cx<double> { using T = dbl2; };

// 1/sqrt(x) for a positive normal x (the callers guarantee it).  Double:
// the hardware estimate refined by one Newton step with its second-order
// term, y (1 + e/2 + 3e^2/8), e = 1 - x y^2.
__device__ __forceinline__ float rsq(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsq(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// Local maximisation of eqs. (4)-(5) in the eq. (3) convention: from the
// staple S, g <- S/|S| (RELAX, omega = 1) or the over-relaxed
// g <- N((1 - omega) g + omega S/|S|), N(v) = v/|v| (for |g| = 1 the same
// map as g N(1 + omega (conj(g) S/|S| - 1))).  |S| = 0 leaves g unchanged.
// Written without branches so that the compiler can schedule a whole colour
// pass as one block.  GUARD keeps the reciprocal square root's argument
// finite at |S| = 0; unguarded, that case runs through infinities and NaNs
// that the final select discards, with the same result and two selects
// fewer (taken where the kernel's register allocation stays spill-free).
// The squared moduli are written as explicit FMAs so that every kernel
// variant rounds them alike.
template <bool RELAX, typename R, bool GUARD = true>
__device__ __forceinline__ typename cx<R>::T local_update(typename cx<R>::T g0, typename cx<R>::T s, R omega)
{
    using C = typename cx<R>::T;
    const R n2 = fma(s.y, s.y, s.x * s.x);
    const bool ok = n2 > (R)0;
    const R r = rsq(GUARD ? (ok ? n2 : (R)1) : n2);
    C g;
    if (RELAX) {
        g.x = s.x * r;
        g.y = s.y * r;
    } else {
        const R a = (R)1 - omega;
        const R b = omega * r;
        const R vx = fma(s.x, b, a * g0.x);
        const R vy = fma(s.y, b, a * g0.y);
        const R rv = rsq(fma(vy, vy, vx * vx));
        g.x = vx * rv;
        g.y = vy * rv;
    }
    g.x = ok ? g.x : g0.x;
    g.y = ok ? g.y : g0.y;
    return g;
}

// Per-start bookkeeping shared by the relax kernels (one lane calls).
__device__ __forceinline__ void record_relax(const GcJobDev &J, uint64_t local, int status, uint64_t sw32,
                                             uint64_t sw64, double D)
{
    GcStartRec r = {};
    r.status = status;
    r.sweeps32 = (uint32_t)sw32;
    r.sweeps64 = (uint32_t)sw64;
    r.D = D;
    r.lambda2 = NAN;
    J.rec[local] = r;
    atomicAdd(&J.cnt->starts_done, 1ULL);
    atomicAdd(status == GC_ST_CONVERGED ? &J.cnt->converged : &J.cnt->nonconverged, 1ULL);
    atomicAdd(&J.cnt->sweeps_total, (unsigned long long)(sw32 + sw64));
}

}  // namespace gc
