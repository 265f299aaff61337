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
#pragma once

#include "gc_common.h"
#include "gc_wave.h"

namespace {

using namespace gc;

// Neighbour half indices of a slot, forward mu = 0..d-1 then backward:
// from its packed table entry (eight 16-bit half indices) ...
struct NbWords {
    u32x4 w;
    __device__ __forceinline__ uint32_t operator()(int k) const
    {
        const uint32_t word = (k >> 1) == 0 ? w.x : (k >> 1) == 1 ? w.y : (k >> 1) == 2 ? w.z : w.w;
        return (k & 1) ? (word >> 16) : (word & 0xFFFFu);
    }
};

// Raw buffer access to a link table: the per-lane byte offset in a VGPR,
// the wave-uniform plane offset in an SGPR, no address arithmetic on the
// vector unit.  Reads past the table's end return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename C> __device__ __forceinline__ C buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ dbl2 buffer_load<dbl2>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <> __device__ __forceinline__ flt2 buffer_load<flt2>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(flt2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// Byte offset of neighbour k in a scaled table entry (16 h per neighbour).
__device__ __forceinline__ uint32_t nb_off(const u32x4 &w, int k)
{
    const uint32_t word = (k >> 1) == 0 ? w.x : (k >> 1) == 1 ? w.y : (k >> 1) == 2 ? w.z : w.w;
    return (k & 1) ? (word >> 16) : (word & 0xFFFFu);
}

// S = sum_k coef_k g_{n_k}, forward mu = 0..d-1 then backward, as in the
// coefficient table, each complex product accumulated by four FMAs.  The
// coefficients come from cf (registers, CF_REG) or from the table at
// coef[(c 2d + k) half + h].
template <int D, typename R, bool CF_REG, typename CP, typename SP, typename NB>
__device__ __forceinline__ typename cx<R>::T staple(const typename cx<R>::T (&cf)[2 * D], CP coef, SP other,
                                                    const NB &nb, int c, int h, int half)
{
    using C = typename cx<R>::T;
    R ax = 0, ay = 0;
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        const C u = CF_REG ? cf[k] : coef[(c * 2 * D + k) * half + h];
        const C g = other[nb(k)];
        ax = fma(u.x, g.x, ax);
        ax = fma(-u.y, g.y, ax);
        ay = fma(u.x, g.y, ay);
        ay = fma(u.y, g.x, ay);
    }
    C s;
    s.x = ax;
    s.y = ay;
    return s;
}

// Synchronisation and reductions over the WPS wavefronts that share a start
// (WPS = 1: one wavefront; otherwise the whole workgroup).  red holds at
// least WPS doubles of LDS.
template <int WPS> __device__ __forceinline__ void start_sync()
{
    if constexpr (WPS > 1) __syncthreads();
    else wave_sync();
}
template <int WPS> __device__ __forceinline__ double start_sum(double v, double *red)
{
    v = wave_sum(v);
    if constexpr (WPS > 1) {
        __syncthreads();   // every wave has read the previous contents of red
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = red[0];
#pragma unroll
        for (int w = 1; w < WPS; ++w) t += red[w];
        v = t;
    }
    return v;
}
template <int WPS> __device__ __forceinline__ double start_max(double v, double *red)
{
    v = wave_max(v);
    if constexpr (WPS > 1) {
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = red[0];
#pragma unroll
        for (int w = 1; w < WPS; ++w) t = fmax(t, red[w]);
        v = t;
    }
    return v;
}

// Sweeps of one precision on the wave's state st[2][half], at most two slots
// per lane (NS <= 2).  Returns status.  Lane l owns slots h = l + 64k, k < NS,
// of each colour; slots beyond the half volume are computed on a clamped
// index and discarded, so the passes have no divergent branches.  The packed
// neighbour entries and the lane's own values are held in registers, and
// CREG colours (0, 1 or 2, starting with colour 0) keep the coefficients of
// the lane's slots in registers for the whole phase.  Colour 0 of sweep
// t + 1 first reads the colour-0 staples of the state after sweep t; at a
// check point they complete the norm of sweep t.
template <int D, typename R, int NS, bool RELAX, bool MAXABS, bool FULL, int CREG, int WPS, typename CP>
__device__ int relax_wave_t(const GcJobDev &J, const GcWaveOrbit &WO, CP coef, lds_ptr<const u32x4> nbt,
                            lds_ptr<typename cx<R>::T> st, double eps, uint64_t cap, bool fixed, uint64_t &sweeps,
                            double &D_out, double *red)
{
    static_assert(NS <= 2, "register-held neighbour entries");
    const int half = WO.half;
    using C = typename cx<R>::T;
    // thread index within the start: the lane, or the workgroup thread when
    // WPS wavefronts share the start
    const int lane = WPS > 1 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    lds_ptr<C> st0 = st;
    lds_ptr<C> st1 = st + half;
    const R omega = (R)J.omega;
    // fixed (batch-synchronous pass): the norm only after the last of cap sweeps
    const uint64_t check = fixed ? cap : J.check_every > 0 ? (uint64_t)J.check_every : 1;
    constexpr bool maxabs = MAXABS;
    int hs[NS];
    bool valid[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int h = lane + 64 * WPS * k;
        valid[k] = FULL || h < half;
        hs[k] = valid[k] ? h : half - 1;
    }
    u32x4 nr[2][NS];
    C own[2][NS];   // the lane's own sites: LDS is only written
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        nr[0][k] = nbt[hs[k]];
        nr[1][k] = nbt[half + hs[k]];
        own[0][k] = st0[hs[k]];
        own[1][k] = st1[hs[k]];
    }
    constexpr int NCR = CREG > 0 ? CREG : 1;
    C cr[NCR][NS][2 * D];
    if constexpr (CREG > 0) {
#pragma unroll
        for (int c = 0; c < CREG; ++c)
#pragma unroll
            for (int k = 0; k < NS; ++k)
#pragma unroll
                for (int q = 0; q < 2 * D; ++q) cr[c][k][q] = coef[(c * 2 * D + q) * half + hs[k]];
    }

    uint64_t t = 0;
    uint64_t until = check;      // sweeps left to the next check point
    bool ckpt = false;           // the state after sweep t is checked
    double part1 = 0.0;          // this lane's colour-1 part of the norm of sweep t
    int status = GC_ST_NONCONVERGED;
    D_out = INFINITY;
    for (;;) {
        const bool pending = (t > 0) && ckpt;
        const bool last = (t == cap);
        // an opaque offset keeps per-slot index arithmetic inside the sweep
        const int z = opaque_zero();
        C gnew[NS];
        double acc0 = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int h = hs[k] + z;
            const C s = staple<D, R, (CREG >= 1)>(cr[0][k], coef, st1, NbWords{nr[0][k]}, 0, h, half);
            const C g0 = own[0][k];
            const double dv = (double)fma(g0.x, s.y, -(g0.y * s.x));
            const double a = maxabs ? fmax(acc0, fabs(dv)) : fma(dv, dv, acc0);
            acc0 = valid[k] ? a : acc0;
            gnew[k] = local_update<RELAX, R, !FULL>(g0, s, omega);
        }
        if (pending) {
            // one wave reduction per checked sweep, over both colours' lane parts
            double Dn;
            if (maxabs) Dn = start_max<WPS>(fmax(acc0, part1), red);
            else Dn = start_sum<WPS>(acc0 + part1, red) / (double)(2 * half);
            D_out = Dn;
            if (!(Dn == Dn)) { status = GC_ST_BADNUM; break; }
            if (Dn < eps) {
                status = GC_ST_CONVERGED;
                if (!fixed) break;
            }
        }
        if (last) break;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            own[0][k] = gnew[k];
            if (valid[k]) st0[hs[k]] = gnew[k];
        }
        start_sync<WPS>();
        // ---- colour 1, with its part of the norm of this sweep
        ++t;
        --until;
        ckpt = (until == 0) || (t == cap);
        if (until == 0) until = check;
        const bool chk = ckpt;
        double a1 = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int h = hs[k] + z;
            const C s = staple<D, R, (CREG >= 2)>(cr[NCR - 1][k], coef, st0, NbWords{nr[1][k]}, 1, h, half);
            const C g = local_update<RELAX, R, !FULL>(own[1][k], s, omega);
            own[1][k] = g;
            if (valid[k]) st1[hs[k]] = g;
            const double dv = (double)fma(g.x, s.y, -(g.y * s.x));
            const double a = maxabs ? fmax(a1, fabs(dv)) : fma(dv, dv, a1);
            a1 = valid[k] ? a : a1;
        }
        if (chk) part1 = a1;
        start_sync<WPS>();
    }
    sweeps = t;
    return status;
}

// Staple of slot h of colour COL from the scaled table entry w: forward
// mu = 0..d-1 then backward, each complex product by four FMAs in the order
// of staple() (a backward coefficient is conj(U), negated exactly).  Table
// offsets are byte offsets of 16-byte sites; the state and the global links
// of single precision have 8-byte sites, hence the shift.  Links of
// directions mu < DL come from LDS planes of lplane bytes holding LT (double
// precision for the double-precision kernel, single precision for the
// single-precision one: the values of the single-precision table), the
// others through buffer loads.  hb: h sizeof(LT).
template <int D, int DL, typename R, typename LT, int COL>
__device__ __forceinline__ typename cx<R>::T staple_big(const u32x4 w, lds_ptr<const unsigned char> other,
                                                        lds_ptr<const unsigned char> lnk, uint32_t hb,
                                                        __amdgpu_buffer_rsrc_t links, uint32_t vo, uint32_t plane,
                                                        uint32_t lplane)
{
    // w holds byte offsets scaled for sites of sizeof(LT) bytes (the
    // single-precision kernel stages the 8-byte table), so offsets of the
    // state and of LDS links need no shift when both are of that size
    using C = typename cx<R>::T;
    constexpr int SH = sizeof(C) == sizeof(LT) ? 0 : (sizeof(C) < sizeof(LT) ? 1 : -1);
    static_assert(SH >= 0, "state sites no larger than link sites");
    constexpr int SHL = 0;
    R ax = 0, ay = 0;
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        const int mu = k < D ? k : k - D;
        const uint32_t raw = nb_off(w, k);
        const uint32_t off = raw >> SH;
        const C g = *(lds_ptr<const C>)(other + off);
        C u;
        if (mu < DL) {
            // [c][mu][slot] planes: own slot or the backward neighbour
            const int c = k < D ? COL : 1 - COL;
            const LT v =
                *(lds_ptr<const LT>)(lnk + (uint32_t)(c * DL + mu) * lplane + (k < D ? hb : (raw >> SHL)));
            u.x = (R)v.x;
            u.y = (R)v.y;
        } else if (k < D) {
            u = buffer_load<C>(links, vo, (uint32_t)(COL * D + mu) * plane);
        } else {
            u = buffer_load<C>(links, off, (uint32_t)((1 - COL) * D + mu) * plane);
        }
        if (k >= D) u.y = -u.y;
        ax = fma(u.x, g.x, ax);
        ax = fma(-u.y, g.y, ax);
        ay = fma(u.x, g.y, ay);
        ay = fma(u.y, g.x, ay);
    }
    C s;
    s.x = ax;
    s.y = ay;
    return s;
}

// The sweep loop specialised per start (uniform branches): plain relaxation
// or over-relaxation, the max |div| or the mean-square norm, and, for the
// double-precision mean-square sweep, whether every slot lies on the lattice
// (half = 64 WPS NS: no slot is tested and the local update skips the guard
// on the reciprocal square root's argument; the single-precision sweep
// measured slower in that form and keeps the general one).  The variants
// round alike.
template <int D, typename R, int NS, int CREG, int WPS, typename CP>
__device__ int relax_wave(const GcJobDev &J, const GcWaveOrbit &WO, CP coef, lds_ptr<const u32x4> nbt,
                          lds_ptr<typename cx<R>::T> st, double eps, uint64_t cap, bool fixed, uint64_t &sweeps,
                          double &D_out, double *red)
{
#define GC_RW(RELAX, MAXABS, FULL)                                                                         \
    return relax_wave_t<D, R, NS, RELAX, MAXABS, FULL, CREG, WPS>(J, WO, coef, nbt, st, eps, cap, fixed, sweeps, \
                                                                  D_out, red)
    const bool relax = (R)J.omega == (R)1;
    if (J.stop_norm != 0) {
        if (relax) GC_RW(true, true, false);
        GC_RW(false, true, false);
    }
    if (sizeof(R) == 8 && WO.half == 64 * WPS * NS) {
        if (relax) GC_RW(true, false, true);
        GC_RW(false, false, true);
    }
    if (relax) GC_RW(true, false, false);
    GC_RW(false, false, false);
#undef GC_RW
}

template <int D, int NS, int CREG, int WPS, typename CP64, typename CP32>
__device__ void relax_start_wave(const GcJobDev &J, const GcWaveOrbit &WO, CP64 coef64, CP32 coef32,
                                 lds_ptr<const u32x4> nbt, lds_ptr<dbl2> st64, lds_ptr<flt2> st32,
                                 glb_ptr<flt2> bounce, uint64_t local, double *red)
{
    constexpr int T = 64 * WPS;   // threads on the start
    const int lane = WPS > 1 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    const GcOrbitDev &O = J.orb;
    const int V = O.V;
    const uint64_t sid = J.first_start + local;

    // random start, written at its colour-split position loc[i]
    for (int b = lane; 4 * b < V; b += T) {
        uint64_t c[4];
        // the caller's start angles, else Philox (the block is skipped then)
        if (!J.theta_init) start_block(J.start_seed, sid, O.orbit_index, (uint64_t)b, c);
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            const int i = 4 * b + k;
            if (i < V) {
                double sn, cs;
                sincos(J.theta_init ? J.theta_init[local * (uint64_t)V + i] : angle_of(c[k]), &sn, &cs);
                const int p = WO.loc[i];
                if (J.precision == 1) st32[p] = flt2{(float)cs, (float)sn};
                else st64[p] = dbl2{cs, sn};
            }
        }
    }
    start_sync<WPS>();

    uint64_t sw32 = 0, sw64 = 0;
    double Dn = INFINITY;
    int status;
    bool in64 = J.precision != 1;
    const bool fixed = (J.flags & GC_JOB_SYNC2) != 0;
    const uint64_t cap = fixed ? (uint64_t)J.fixed_sweeps[local] : J.max_sweeps;
    if (J.precision == 1) {
        status = relax_wave<D, float, NS, CREG, WPS>(J, WO, coef32, nbt, st32, J.eps32, J.max_sweeps, false, sw32, Dn,
                                                     red);
        if (status == GC_ST_CONVERGED) {
            // promotion g64 = normalise((double) g32): both states share the
            // start's LDS region, so each thread bounces its entries through
            // the start's scratch (it reads back only what it wrote)
            in64 = true;
            for (int p = lane; p < V; p += T) bounce[p] = st32[p];
            start_sync<WPS>();
            for (int p = lane; p < V; p += T) {
                const flt2 g = bounce[p];
                const double xr = (double)g.x, xi = (double)g.y;
                const double r = rsqrt(xr * xr + xi * xi);
                st64[p] = dbl2{xr * r, xi * r};
            }
            start_sync<WPS>();
            status = relax_wave<D, double, NS, CREG, WPS>(J, WO, coef64, nbt, st64, J.eps64, J.max_sweeps, false,
                                                          sw64, Dn, red);
        }
    } else {
        status = relax_wave<D, double, NS, CREG, WPS>(J, WO, coef64, nbt, st64, J.eps64, cap, fixed, sw64, Dn, red);
    }
    // final state in natural site order
    glb_ptr<dbl2> out = as_global(reinterpret_cast<dbl2 *>(J.states + local * (uint64_t)V));
    for (int i = lane; i < V; i += T) {
        const int p = WO.loc[i];
        out[i] = in64 ? st64[p] : dbl2{(double)st32[p].x, (double)st32[p].y};
    }
    if (lane == 0) record_relax(J, local, status, sw32, sw64, Dn);
    start_sync<WPS>();
}

// Exchange-region variant for more than two slots per lane (NS > 2).  A
// start keeps one region X[half] in LDS, holding the colour that the next
// pass reads; the lane holds the values of its own slots of the colour being
// updated in registers.  Colour-0 pass: staples from X (colour 1), new
// values into registers (kept until the stopping norm of the previous sweep
// has been decided); then every lane takes its colour-1 values back from X
// and writes its new colour-0 values in their place.  Colour-1 pass:
// staples from X (colour 0), values updated in registers; then the lanes
// swap colour 0 back out of X and colour 1 in.  One wavefront runs a start
// alone, so the LDS instructions of a pass (all reads, then the swap) are
// ordered by program order; the fences keep the compiler from moving them.
// Half the LDS of a two-region state lets twice the starts share a compute
// unit.  The sweep schedule, the stopping norm and the arithmetic are those
// of relax_wave_t.  own: the start's values on entry and on return.
// Slots beyond the half volume work on the clamped site half - 1 and are
// neither stored nor counted.  FULL: every slot of a lane but its last lies
// on the lattice (ceil(half / 64) = NS), so only the last slot is tested;
// the norm's products are explicit FMAs, so both variants round alike.
template <int D, typename R, int NS, bool RELAX, bool MAXABS, int DL, typename LT, bool FULL = false>
__device__ int relax_rr(const GcJobDev &J, int half, __amdgpu_buffer_rsrc_t links, lds_ptr<const unsigned char> lb,
                        lds_ptr<const u32x4> nbt, lds_ptr<typename cx<R>::T> X, typename cx<R>::T (&own)[2][NS],
                        double eps, uint64_t cap, bool fixed, uint64_t &sweeps, double &D_out)
{
    using C = typename cx<R>::T;
    const int lane = (int)(threadIdx.x & 63);
    lds_ptr<const unsigned char> xb = (lds_ptr<const unsigned char>)X;
    constexpr uint32_t lplane = 64u * NS * (uint32_t)sizeof(LT);   // staged link planes: 64 NS sites each
    const uint32_t plane = (uint32_t)half * (uint32_t)sizeof(C);
    const R omega = (R)J.omega;
    const uint64_t check = fixed ? cap : J.check_every > 0 ? (uint64_t)J.check_every : 1;
    constexpr bool maxabs = MAXABS;
    // slot k of the lane: h = lane + 64 k, computed on a clamped index and
    // discarded beyond the half volume (recomputed where used: no
    // registers held for it)
#define GC_RR_SLOT(k) const int hk = lane + 64 * (k); const bool vk = (FULL && (k) < NS - 1) || hk < half; const int hc = vk ? hk : half - 1
    // the first pass reads colour 1
    wave_sync();
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        GC_RR_SLOT(k);
        (void)hc;
        if (vk) X[hk] = own[1][k];
    }
    wave_sync();
    C g0r[NS], g1r[NS];   // colour-0 values (colour-0 pass), colour-1 values (colour-1 pass)
#pragma unroll
    for (int k = 0; k < NS; ++k) g0r[k] = own[0][k];

    uint64_t t = 0;
    uint64_t until = check;
    bool ckpt = false;
    double part1 = 0.0;
    int status = GC_ST_NONCONVERGED;
    D_out = INFINITY;
    for (;;) {
        const bool pending = (t > 0) && ckpt;
        const bool last = (t == cap);
        const int z = opaque_zero();
        C gnew[NS];
        double acc0 = 0.0;
        u32x4 wnext = nbt[min(lane, half - 1) + z];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            GC_RR_SLOT(k);
            const int h = hc + z;
            const u32x4 wcur = wnext;
            if (k + 1 < NS) wnext = nbt[min(lane + 64 * (k + 1), half - 1) + z];
            const C s = staple_big<D, DL, R, LT, 0>(wcur, xb, lb, (uint32_t)h * (uint32_t)sizeof(LT), links,
                                                (uint32_t)h * (uint32_t)sizeof(C), plane, lplane);
            const C g0 = g0r[k];
            const double dv = (double)fma(g0.x, s.y, -(g0.y * s.x));
            const double a = maxabs ? fmax(acc0, fabs(dv)) : fma(dv, dv, acc0);
            acc0 = vk ? a : acc0;
            gnew[k] = local_update<RELAX, R, !FULL>(g0, s, omega);
        }
        if (pending) {
            double Dn;
            if (maxabs) Dn = wave_max(fmax(acc0, part1));
            else Dn = wave_sum(acc0 + part1) / (double)(2 * half);
            D_out = Dn;
            if (!(Dn == Dn)) { status = GC_ST_BADNUM; break; }
            if (Dn < eps) {
                status = GC_ST_CONVERGED;
                if (!fixed) break;
            }
        }
        if (last) break;
        // swap: colour 1 out of X, the new colour 0 in
        wave_sync();
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            GC_RR_SLOT(k);
            g1r[k] = X[hc];
            if (vk) X[hk] = gnew[k];
        }
        wave_sync();
        ++t;
        --until;
        ckpt = (until == 0) || (t == cap);
        if (until == 0) until = check;
        const bool chk = ckpt;
        double a1 = 0.0;
        u32x4 wnext1 = nbt[half + min(lane, half - 1) + z];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            GC_RR_SLOT(k);
            const int h = hc + z;
            const u32x4 wcur = wnext1;
            if (k + 1 < NS) wnext1 = nbt[half + min(lane + 64 * (k + 1), half - 1) + z];
            const C s = staple_big<D, DL, R, LT, 1>(wcur, xb, lb, (uint32_t)h * (uint32_t)sizeof(LT), links,
                                                (uint32_t)h * (uint32_t)sizeof(C), plane, lplane);
            const C g = local_update<RELAX, R, !FULL>(g1r[k], s, omega);
            g1r[k] = g;
            const double dv = (double)fma(g.x, s.y, -(g.y * s.x));
            const double a = maxabs ? fmax(a1, fabs(dv)) : fma(dv, dv, a1);
            a1 = vk ? a : a1;
        }
        if (chk) part1 = a1;
        // swap: colour 0 out of X, the new colour 1 in
        wave_sync();
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            GC_RR_SLOT(k);
            g0r[k] = X[hc];
            if (vk) X[hk] = g1r[k];
        }
        wave_sync();
    }
    // X holds colour 1
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        GC_RR_SLOT(k);
        (void)vk;
        own[0][k] = g0r[k];
        own[1][k] = X[hc];
    }
    wave_sync();
#undef GC_RR_SLOT
    sweeps = t;
    return status;
}

// Relax modes of the exchange-region kernel, fixed per launch from omega:
// over-relaxation in both precisions, plain relaxation in both (omega = 1),
// or plain relaxation in the single-precision phase only (omega rounds to 1
// in single precision but differs from 1); GC_RM_MAXABS added for the
// max |div| stopping norm; GC_RM_FULL (double-precision kernel) where every
// orbit of the launch has ceil(half / 64) = NS.
enum { GC_RM_OR = 0, GC_RM_RELAX = 1, GC_RM_RELAX32 = 2, GC_RM_MAXABS = 4, GC_RM_FULL = GC_RM_FULL_SLOTS };

template <int D, typename R, int NS, bool RELAX, bool MAXABS, int DL, typename LT, bool FULL = false>
__device__ __forceinline__ int relax_rr_links(const GcJobDev &J, const GcWaveOrbit &WO,
                                              lds_ptr<const unsigned char> lnk, lds_ptr<const u32x4> nbt,
                                              lds_ptr<typename cx<R>::T> X, typename cx<R>::T (&own)[2][NS],
                                              double eps, uint64_t cap, bool fixed, uint64_t &sweeps, double &D_out)
{
    const uint32_t bytes = (uint32_t)(2 * D * WO.half * sizeof(typename cx<R>::T));
    const __amdgpu_buffer_rsrc_t links =
        buffer_rsrc(sizeof(R) == 8 ? (const void *)WO.link64 : (const void *)WO.link32, bytes);
    return relax_rr<D, R, NS, RELAX, MAXABS, DL, LT, FULL>(J, WO.half, links, lnk, nbt, X, own, eps, cap, fixed,
                                                           sweeps, D_out);
}

// The links of the first DL directions, both colours, into LDS planes of
// 64 NS sites (plane c DL + mu) from the [c][mu][half] table src.
template <int D, int NS, int DL, typename LT>
__device__ __forceinline__ void rr_stage_links(lds_ptr<LT> lnk, const LT *src, int half, int nthreads)
{
    if constexpr (DL > 0) {
        glb_ptr<const LT> lg = as_global(src);
        for (int t = threadIdx.x; t < 2 * DL * half; t += nthreads) {
            const int pl = t / half, h = t - pl * half;
            const int c = pl / DL, mu = pl - c * DL;
            lnk[pl * 64 * NS + h] = lg[(c * D + mu) * half + h];
        }
    }
}

// Final state in natural site order, one colour per round through X.
template <int NS>
__device__ __forceinline__ void rr_store(const GcJobDev &J, const GcWaveOrbit &WO, lds_ptr<dbl2> X64, uint64_t local,
                                         const dbl2 (&own64)[2][NS])
{
    const int lane = (int)(threadIdx.x & 63);
    const int V = J.orb.V, half = WO.half;
    glb_ptr<dbl2> out = as_global(reinterpret_cast<dbl2 *>(J.states + local * (uint64_t)V));
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        wave_sync();
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int h = lane + 64 * k;
            if (h < half) X64[h] = own64[c][k];
        }
        wave_sync();
        for (int i = lane; i < V; i += 64) {
            const int p = WO.loc[i] - c * half;
            if (p >= 0 && p < half) out[i] = X64[p];
        }
    }
    wave_sync();
}

// Values of colour c of a start, exchanged through X: slot h of the lane's
// own list, from the sites i with loc[i] = c half + h.
template <typename C, int NS>
__device__ __forceinline__ void rr_gather(lds_ptr<C> X, C (&dst)[NS], int half)
{
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int h = lane + 64 * k;
        dst[k] = X[h < half ? h : half - 1];
    }
}

template <int D, int NS, typename C>
__device__ __forceinline__ void rr_init(const GcJobDev &J, const GcWaveOrbit &WO, lds_ptr<C> X, uint64_t local,
                                        C (&own)[2][NS])
{
    const int lane = (int)(threadIdx.x & 63);
    const GcOrbitDev &O = J.orb;
    const int V = O.V;
    const int half = WO.half;
    const uint64_t sid = J.first_start + local;
    // random start (or the caller's angles), one colour per round: the sites
    // of colour c go to X at their half index, then to the lanes' slots
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        wave_sync();
        for (int b = lane; 4 * b < V; b += 64) {
            uint64_t w[4];
            if (!J.theta_init) start_block(J.start_seed, sid, O.orbit_index, (uint64_t)b, w);
#pragma unroll 1
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * b + q;
                if (i < V) {
                    const int p = WO.loc[i] - c * half;
                    if (p >= 0 && p < half) {
                        double sn, cs;
                        sincos(J.theta_init ? J.theta_init[local * (uint64_t)V + i] : angle_of(w[q]), &sn, &cs);
                        if constexpr (sizeof(C) == 8) X[p] = flt2{(float)cs, (float)sn};
                        else X[p] = dbl2{cs, sn};
                    }
                }
            }
        }
        wave_sync();
        rr_gather<C, NS>(X, own[c], half);
    }
}

// One start on the double-precision exchange-region kernel: from the random
// (or given) angles, or, for a mixed launch (GC_JOB_FROM32), from the state
// the single-precision kernel promoted to HBM; starts that the
// single-precision kernel finished (not converged) are skipped.
template <int D, int NS, int RM>
__device__ void relax_start_rr(const GcJobDev &J, const GcWaveOrbit &WO, lds_ptr<const unsigned char> lnk,
                               lds_ptr<const u32x4> nbt, lds_ptr<unsigned char> xr, uint64_t local)
{
    const int lane = (int)(threadIdx.x & 63);
    const int V = J.orb.V;
    const int half = WO.half;
    lds_ptr<dbl2> X64 = (lds_ptr<dbl2>)xr;
    dbl2 own64[2][NS];
    uint64_t sw32 = 0, sw64 = 0;
    double Dn = INFINITY;
    const bool from32 = (J.flags & GC_JOB_FROM32) != 0;
    if (from32) {
        const GcStartRec r = J.rec[local];
        if (r.status != GC_ST_PROMOTED) return;   // finished in single precision
        sw32 = r.sweeps32;
        // the promoted state, natural site order, one colour per round
        glb_ptr<const dbl2> in = as_global(reinterpret_cast<const dbl2 *>(J.states + local * (uint64_t)V));
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            wave_sync();
            for (int i = lane; i < V; i += 64) {
                const int p = WO.loc[i] - c * half;
                if (p >= 0 && p < half) X64[p] = in[i];
            }
            wave_sync();
            rr_gather<dbl2, NS>(X64, own64[c], half);
        }
    } else {
        rr_init<D, NS, dbl2>(J, WO, X64, local, own64);
    }
    const bool fixed = !from32 && (J.flags & GC_JOB_SYNC2) != 0;
    const uint64_t cap = fixed ? (uint64_t)J.fixed_sweeps[local] : J.max_sweeps;
    const int status =
        relax_rr_links<D, double, NS, (RM & 3) == GC_RM_RELAX, (RM & GC_RM_MAXABS) != 0, gc_links_in_lds(D, NS), dbl2,
                       (RM & GC_RM_FULL) != 0>(J, WO, lnk, nbt, X64, own64, J.eps64, cap, fixed, sw64, Dn);
    rr_store<NS>(J, WO, X64, local, own64);
    if (lane == 0) record_relax(J, local, status, sw32, sw64, Dn);
    wave_sync();
}

// One start on the single-precision kernel of a mixed launch: relaxed to
// eps32, then either promoted (g64 = normalise((double) g32)) into HBM for
// the double-precision kernel, or, not converged, finished here with its
// single-precision values widened.
template <int D, int NS, int RM>
__device__ void relax_start_rr32(const GcJobDev &J, const GcWaveOrbit &WO, lds_ptr<const unsigned char> lnk,
                                 lds_ptr<const u32x4> nbt, lds_ptr<unsigned char> xr, uint64_t local)
{
    const int lane = (int)(threadIdx.x & 63);
    const int V = J.orb.V;
    const int half = WO.half;
    lds_ptr<flt2> X32 = (lds_ptr<flt2>)xr;
    flt2 own32[2][NS];
    uint64_t sw32 = 0;
    double Dn = INFINITY;
    rr_init<D, NS, flt2>(J, WO, X32, local, own32);
    const int status =
        relax_rr_links<D, float, NS, (RM & 3) != GC_RM_OR, (RM & GC_RM_MAXABS) != 0, gc_links_in_lds32(D, NS), flt2>(
            J, WO, lnk, nbt, X32, own32, J.eps32, J.max_sweeps, false, sw32, Dn);
    const bool conv = status == GC_ST_CONVERGED;
    // natural site order, one colour per round through X (single precision)
    glb_ptr<dbl2> out = as_global(reinterpret_cast<dbl2 *>(J.states + local * (uint64_t)V));
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        wave_sync();
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int h = lane + 64 * k;
            if (h < half) X32[h] = own32[c][k];
        }
        wave_sync();
        for (int i = lane; i < V; i += 64) {
            const int p = WO.loc[i] - c * half;
            if (p >= 0 && p < half) {
                const flt2 g = X32[p];
                const double xr_ = (double)g.x, xi = (double)g.y;
                const double r = conv ? rsqrt(xr_ * xr_ + xi * xi) : 1.0;
                out[i] = dbl2{xr_ * r, xi * r};
            }
        }
    }
    wave_sync();
    if (lane == 0) {
        if (conv) {
            GcStartRec r = {};
            r.status = GC_ST_PROMOTED;
            r.sweeps32 = (uint32_t)sw32;
            r.D = Dn;
            r.lambda2 = NAN;
            J.rec[local] = r;
        } else {
            record_relax(J, local, status, sw32, 0, Dn);
        }
    }
    wave_sync();
}

// WG = WAVES wavefronts, at most two slots per lane.  LDS: [neighbour table
// 16V | coef64 | coef32 when COEF_LDS] then per wave a 16V-byte state region
// (double2[V], or float2[V] in the single-precision phase).
template <int D, int NS, int WAVES, bool COEF_LDS, int CREG>
__global__ __launch_bounds__(64 * WAVES) void wave_kernel(const GcJobDev *__restrict__ jobs,
                                                          const GcWaveOrbit *__restrict__ worbs, int n_jobs,
                                                          unsigned long long *job_next, float2 *bounce_all)
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
        const int jn = uniform(cur_job);
        __syncthreads();
        if (jn < 0) break;
        const GcJobDev &J = jobs[jn];
        const GcWaveOrbit &WO = worbs[jn];
        const int V = J.orb.V;
        const int ncoef = 2 * D * V;      // complex entries per precision
        // neighbour table (16 bytes per slot, 16V in all), then the
        // coefficients when staged, then the wavefronts' states
        lds_ptr<u32x4> nbt = as_lds(reinterpret_cast<u32x4 *>(smem));
        {
            glb_ptr<const u32x4> nbg = as_global(reinterpret_cast<const u32x4 *>(WO.nb));
            for (int t = threadIdx.x; t < V; t += 64 * WAVES) nbt[t] = nbg[t];
        }
        size_t off = 16 * (size_t)V;
        const dbl2 *g64 = reinterpret_cast<const dbl2 *>(WO.coef64);
        const flt2 *g32 = reinterpret_cast<const flt2 *>(WO.coef32);
        lds_ptr<dbl2> c64 = as_lds(reinterpret_cast<dbl2 *>(smem + off));
        lds_ptr<flt2> c32 = as_lds(reinterpret_cast<flt2 *>(smem + off + 16 * (size_t)ncoef));
        if (COEF_LDS) {
            for (int t = threadIdx.x; t < ncoef; t += 64 * WAVES) c64[t] = g64[t];
            off += 16 * (size_t)ncoef;
            if (J.precision == 1) {
                for (int t = threadIdx.x; t < ncoef; t += 64 * WAVES) c32[t] = g32[t];
                off += 8 * (size_t)ncoef;
            }
        }
        __syncthreads();
        lds_ptr<dbl2> st64 = as_lds(reinterpret_cast<dbl2 *>(smem + off + (size_t)wave * 16 * V));
        lds_ptr<flt2> st32 = as_lds(reinterpret_cast<flt2 *>(smem + off + (size_t)wave * 16 * V));
        glb_ptr<flt2> bounce =
            as_global(reinterpret_cast<flt2 *>(bounce_all) + ((uint64_t)blockIdx.x * WAVES + wave) * (uint64_t)V);
        for (;;) {
            unsigned long long s = 0;
            if (lane == 0) s = atomicAdd(&job_next[jn], 1ULL);
            s = uniform((uint64_t)s);
            if (s >= J.n_starts) break;
            lds_ptr<const u32x4> nbc = nbt;
            if (COEF_LDS)
                relax_start_wave<D, NS, CREG, 1>(J, WO, c64, c32, nbc, st64, st32, bounce, s, nullptr);
            else
                relax_start_wave<D, NS, CREG, 1>(J, WO, as_global(g64), as_global(g32), nbc, st64, st32, bounce, s,
                                                 nullptr);
        }
        __syncthreads();
        j0 = jn;
    }
}

// WG = GC_WAVES_RR wavefronts, one start each, for lattices with more than
// two slots per lane, double precision.  LDS (gc_rr_lds_bytes): [links of DL
// directions, planes of 64 NS double2 | neighbour table 16V (byte offsets)]
// then per wave an 8V-byte exchange region (double2[half]).
template <int D, int NS, int RM>
__global__ __launch_bounds__(64 * GC_WAVES_RR) void wave_rr_kernel(const GcJobDev *__restrict__ jobs,
                                                                    const GcWaveOrbit *__restrict__ worbs,
                                                                    int n_jobs, unsigned long long *job_next)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cur_job;
    constexpr int DL = gc_links_in_lds(D, NS);
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
        const int jn = uniform(cur_job);
        __syncthreads();
        if (jn < 0) break;
        const GcJobDev &J = jobs[jn];
        const GcWaveOrbit &WO = worbs[jn];
        const int V = J.orb.V;
        const int half = WO.half;
        constexpr size_t LB = gc_rr_links_bytes(D, NS);
        rr_stage_links<D, NS, DL, dbl2>(as_lds(reinterpret_cast<dbl2 *>(smem)),
                                        reinterpret_cast<const dbl2 *>(WO.link64), half, 64 * GC_WAVES_RR);
        lds_ptr<const unsigned char> lnk = as_lds(reinterpret_cast<const unsigned char *>(smem));
        lds_ptr<u32x4> nbt = as_lds(reinterpret_cast<u32x4 *>(smem + LB));
        glb_ptr<const u32x4> nbg = as_global(reinterpret_cast<const u32x4 *>(WO.nbo));
        for (int t = threadIdx.x; t < V; t += 64 * GC_WAVES_RR) nbt[t] = nbg[t];
        __syncthreads();
        lds_ptr<unsigned char> xr = as_lds(smem + LB + 16 * (size_t)V + (size_t)wave * 8 * V);
        for (;;) {
            unsigned long long s = 0;
            if (lane == 0) s = atomicAdd(&job_next[jn], 1ULL);
            s = uniform((uint64_t)s);
            if (s >= J.n_starts) break;
            relax_start_rr<D, NS, RM>(J, WO, lnk, nbt, xr, s);
        }
        __syncthreads();
        j0 = jn;
    }
}

// WG = GC_WAVES_RR32 wavefronts, one start each: the single-precision phase
// of mixed launches with more than two slots per lane.  LDS
// (gc_rr32_lds_bytes): [links of DL directions, planes of 64 NS float2 |
// neighbour table 16V] then per wave a 4V-byte exchange region (float2[half]).
template <int D, int NS, int RM>
__global__ __launch_bounds__(64 * GC_WAVES_RR32) void wave_rr32_kernel(const GcJobDev *__restrict__ jobs,
                                                                        const GcWaveOrbit *__restrict__ worbs,
                                                                        int n_jobs, unsigned long long *job_next)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cur_job;
    constexpr int DL = gc_links_in_lds32(D, NS);
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
        const int jn = uniform(cur_job);
        __syncthreads();
        if (jn < 0) break;
        const GcJobDev &J = jobs[jn];
        const GcWaveOrbit &WO = worbs[jn];
        const int V = J.orb.V;
        const int half = WO.half;
        constexpr size_t LB = gc_rr32_links_bytes(D, NS);
        rr_stage_links<D, NS, DL, flt2>(as_lds(reinterpret_cast<flt2 *>(smem)),
                                        reinterpret_cast<const flt2 *>(WO.link32), half, 64 * GC_WAVES_RR32);
        lds_ptr<const unsigned char> lnk = as_lds(reinterpret_cast<const unsigned char *>(smem));
        lds_ptr<u32x4> nbt = as_lds(reinterpret_cast<u32x4 *>(smem + LB));
        glb_ptr<const u32x4> nbg = as_global(reinterpret_cast<const u32x4 *>(WO.nbo32));
        for (int t = threadIdx.x; t < V; t += 64 * GC_WAVES_RR32) nbt[t] = nbg[t];
        __syncthreads();
        lds_ptr<unsigned char> xr = as_lds(smem + LB + 16 * (size_t)V + (size_t)wave * 4 * V);
        for (;;) {
            unsigned long long s = 0;
            if (lane == 0) s = atomicAdd(&job_next[jn], 1ULL);
            s = uniform((uint64_t)s);
            if (s >= J.n_starts) break;
            relax_start_rr32<D, NS, RM>(J, WO, lnk, nbt, xr, s);
        }
        __syncthreads();
        j0 = jn;
    }
}

template <int D, int NS, int WAVES>
hipError_t launch32_t(const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs, unsigned long long *job_next,
                      int rm, int grid, size_t lds, hipStream_t s)
{
    if constexpr (NS > 2) {
        switch (rm) {
#define GC_RR32_LAUNCH(RM)                                                                                \
    case RM:                                                                                              \
        hipLaunchKernelGGL((wave_rr32_kernel<D, NS, RM>), dim3(grid), dim3(64 * GC_WAVES_RR32), lds, s, jobs,  \
                           worbs, n_jobs, job_next);                                                      \
        break;
            GC_RR32_LAUNCH(0)
            GC_RR32_LAUNCH(1)
            GC_RR32_LAUNCH(2)
            GC_RR32_LAUNCH(4)
            GC_RR32_LAUNCH(5)
            GC_RR32_LAUNCH(6)
#undef GC_RR32_LAUNCH
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <int D, int NS, int WAVES>
hipError_t occ32_t(int rm, size_t lds, int *per_cu)
{
    (void)rm;
    if constexpr (NS > 2)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, wave_rr32_kernel<D, NS, GC_RM_OR>,
                                                            64 * GC_WAVES_RR32, lds);
    else
        return hipErrorInvalidValue;
}

// One start per workgroup of WPS wavefronts, for lattices with more than 128
// slots per colour: each thread keeps at most two slots per colour, the
// colour passes synchronise the workgroup.  LDS: the neighbour table (16V)
// and one state region (16V); the coefficients are read from global memory.
template <int D, int WPS>
__global__ __launch_bounds__(64 * WPS) void wps_kernel(const GcJobDev *__restrict__ jobs,
                                                       const GcWaveOrbit *__restrict__ worbs, int n_jobs,
                                                       unsigned long long *job_next, float2 *bounce_all)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cur_job;
    __shared__ unsigned long long claim;
    __shared__ double red[WPS];
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
        const int jn = uniform(cur_job);
        __syncthreads();
        if (jn < 0) break;
        const GcJobDev &J = jobs[jn];
        const GcWaveOrbit &WO = worbs[jn];
        const int V = J.orb.V;
        lds_ptr<u32x4> nbt = as_lds(reinterpret_cast<u32x4 *>(smem));
        glb_ptr<const u32x4> nbg = as_global(reinterpret_cast<const u32x4 *>(WO.nb));
        for (int t = threadIdx.x; t < V; t += 64 * WPS) nbt[t] = nbg[t];
        __syncthreads();
        lds_ptr<dbl2> st64 = as_lds(reinterpret_cast<dbl2 *>(smem + 16 * (size_t)V));
        lds_ptr<flt2> st32 = as_lds(reinterpret_cast<flt2 *>(smem + 16 * (size_t)V));
        glb_ptr<flt2> bounce = as_global(reinterpret_cast<flt2 *>(bounce_all) + (uint64_t)blockIdx.x * (uint64_t)V);
        const dbl2 *g64 = reinterpret_cast<const dbl2 *>(WO.coef64);
        const flt2 *g32 = reinterpret_cast<const flt2 *>(WO.coef32);
        lds_ptr<const u32x4> nbc = nbt;
        for (;;) {
            if (threadIdx.x == 0) claim = atomicAdd(&job_next[jn], 1ULL);
            __syncthreads();
            const uint64_t s = uniform((uint64_t)claim);
            __syncthreads();
            if (s >= J.n_starts) break;
            relax_start_wave<D, 2, 0, WPS>(J, WO, as_global(g64), as_global(g32), nbc, st64, st32, bounce, s, red);
        }
        __syncthreads();
        j0 = jn;
    }
}

template <int D, int WPS>
hipError_t wps_launch_t(const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs, unsigned long long *job_next,
                        float2 *bounce, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((wps_kernel<D, WPS>), dim3(grid), dim3(64 * WPS), lds, s, jobs, worbs, n_jobs, job_next,
                       bounce);
    return hipGetLastError();
}

template <int D, int WPS>
hipError_t wps_occ_t(size_t lds, int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, wps_kernel<D, WPS>, 64 * WPS, lds);
}

template <int D, int NS, int WAVES, bool CL, int CREG>
hipError_t launch_v(const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs, unsigned long long *job_next,
                    float2 *bounce, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((wave_kernel<D, NS, WAVES, CL, CREG>), dim3(grid), dim3(64 * WAVES), lds, s, jobs, worbs,
                       n_jobs, job_next, bounce);
    return hipGetLastError();
}

template <int D, int NS, int WAVES, bool CL, int CREG>
hipError_t occ_v(size_t lds, int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, wave_kernel<D, NS, WAVES, CL, CREG>, 64 * WAVES, lds);
}

// Register-held coefficients are instantiated where a lane's slots are few
// (NS <= 2): creg 1 holds colour 0, creg 2 both colours.
template <int D, int NS> constexpr bool creg_ok() { return NS <= 2; }

template <int D, int NS, int WAVES>
hipError_t launch_t(const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs, unsigned long long *job_next,
                    int variant, float2 *bounce, int grid, size_t lds, hipStream_t s)
{
    const bool cl = (variant & 1) != 0;
    const int creg = (variant >> 1) & 3;
    if constexpr (creg_ok<D, NS>()) {
        if (creg == 1)
            return cl ? launch_v<D, NS, WAVES, true, 1>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s)
                      : launch_v<D, NS, WAVES, false, 1>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);
        if (creg == 2)
            return cl ? launch_v<D, NS, WAVES, true, 2>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s)
                      : launch_v<D, NS, WAVES, false, 2>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);
    }
    if (creg != 0) return hipErrorInvalidValue;
    if constexpr (NS > 2) {
        // register-resident kernel: no staged coefficient table
        if (cl) return hipErrorInvalidValue;
        (void)bounce;
        switch ((variant >> 3) & 15) {
#define GC_RR_LAUNCH(RM)                                                                                  \
    case RM:                                                                                              \
        hipLaunchKernelGGL((wave_rr_kernel<D, NS, RM>), dim3(grid), dim3(64 * GC_WAVES_RR), lds, s, jobs, worbs, \
                           n_jobs, job_next);                                                             \
        break;
            GC_RR_LAUNCH(0)
            GC_RR_LAUNCH(1)
            GC_RR_LAUNCH(2)
            GC_RR_LAUNCH(4)
            GC_RR_LAUNCH(5)
            GC_RR_LAUNCH(6)
            GC_RR_LAUNCH(GC_RM_FULL)
            GC_RR_LAUNCH(GC_RM_FULL | 1)
            GC_RR_LAUNCH(GC_RM_FULL | 2)
            GC_RR_LAUNCH(GC_RM_FULL | 4)
            GC_RR_LAUNCH(GC_RM_FULL | 5)
            GC_RR_LAUNCH(GC_RM_FULL | 6)
#undef GC_RR_LAUNCH
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    } else {
        return cl ? launch_v<D, NS, WAVES, true, 0>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s)
                  : launch_v<D, NS, WAVES, false, 0>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);
    }
}

template <int D, int NS, int WAVES>
hipError_t occ_t(int variant, size_t lds, int *per_cu)
{
    const bool cl = (variant & 1) != 0;
    const int creg = (variant >> 1) & 3;
    if constexpr (creg_ok<D, NS>()) {
        if (creg == 1) return cl ? occ_v<D, NS, WAVES, true, 1>(lds, per_cu) : occ_v<D, NS, WAVES, false, 1>(lds, per_cu);
        if (creg == 2) return cl ? occ_v<D, NS, WAVES, true, 2>(lds, per_cu) : occ_v<D, NS, WAVES, false, 2>(lds, per_cu);
    }
    if (creg != 0) return hipErrorInvalidValue;
    if constexpr (NS > 2) {
        if (cl) return hipErrorInvalidValue;
        // the three relax modes share their resource use; the
        // over-relaxation instantiation stands for them
        if ((variant >> 3) & GC_RM_FULL)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, wave_rr_kernel<D, NS, GC_RM_FULL>,
                                                                64 * GC_WAVES_RR, lds);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, wave_rr_kernel<D, NS, GC_RM_OR>, 64 * GC_WAVES_RR,
                                                            lds);
    } else {
        return cl ? occ_v<D, NS, WAVES, true, 0>(lds, per_cu) : occ_v<D, NS, WAVES, false, 0>(lds, per_cu);
    }
}


}  // namespace

// Entry points of one lattice dimension D: each gc_waveD.hip instantiates
// the kernels of its D only (NS = slots per lane per colour =
// ceil(half / 64), instantiated for half-volumes up to 1024 sites, the
// largest whose states and table fit in LDS).
#define GC_WAVE_DEFINE_DIM(D, NS_LIST)                                                                    \
    hipError_t gc_wave_occupancy_d##D(int ns, int variant, size_t lds, int *per_cu)                        \
    {                                                                                                     \
        NS_LIST(occ_t, D, variant, lds, per_cu)                                                           \
    }                                                                                                     \
    hipError_t gc_launch_wave_d##D(int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,   \
                                   unsigned long long *job_next, int variant, float2 *bounce, int grid,   \
                                   size_t lds, hipStream_t s)                                             \
    {                                                                                                     \
        NS_LIST(launch_t, D, jobs, worbs, n_jobs, job_next, variant, bounce, grid, lds, s)               \
    }                                                                                                     \
    hipError_t gc_wave32_occupancy_d##D(int ns, int rm, size_t lds, int *per_cu)                          \
    {                                                                                                     \
        NS_LIST(occ32_t, D, rm, lds, per_cu)                                                              \
    }                                                                                                     \
    hipError_t gc_launch_wave32_d##D(int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs, \
                                     unsigned long long *job_next, int rm, int grid, size_t lds,          \
                                     hipStream_t s)                                                       \
    {                                                                                                     \
        NS_LIST(launch32_t, D, jobs, worbs, n_jobs, job_next, rm, grid, lds, s)                           \
    }                                                                                                     \
    hipError_t gc_wps_occupancy_d##D(int wps, size_t lds, int *per_cu)                                    \
    {                                                                                                     \
        switch (wps) {                                                                                    \
        case 2: return wps_occ_t<D, 2>(lds, per_cu);                                                      \
        case 4: return wps_occ_t<D, 4>(lds, per_cu);                                                      \
        case 6: return wps_occ_t<D, 6>(lds, per_cu);                                                      \
        case 8: return wps_occ_t<D, 8>(lds, per_cu);                                                      \
        case 16: return wps_occ_t<D, 16>(lds, per_cu);                                                    \
        default: return hipErrorInvalidValue;                                                             \
        }                                                                                                 \
    }                                                                                                     \
    hipError_t gc_launch_wps_d##D(int wps, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,   \
                                  unsigned long long *job_next, float2 *bounce, int grid, size_t lds,     \
                                  hipStream_t s)                                                          \
    {                                                                                                     \
        switch (wps) {                                                                                    \
        case 2: return wps_launch_t<D, 2>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);          \
        case 4: return wps_launch_t<D, 4>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);          \
        case 6: return wps_launch_t<D, 6>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);          \
        case 8: return wps_launch_t<D, 8>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);          \
        case 16: return wps_launch_t<D, 16>(jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);        \
        default: return hipErrorInvalidValue;                                                             \
        }                                                                                                 \
    }
