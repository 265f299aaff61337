// Colour-split tables and launch entry points of the wavefront-per-start
// solver (lattices whose extents are all even).
#pragma once

#include "gc_internal.h"

struct GcWaveOrbit {
    int32_t half, pad;              // V / 2
    const uint16_t *loc;            // [V] site -> c * half + h
    const uint4 *nb;                // [2][half] neighbour half indices, 8 x u16 (forward mu, then backward)
    const double2 *coef64;          // [2][2d][half] U_{i,k} (forward) / conj(U_{i-k,k}) (backward)
    const float2 *coef32;           // same, rounded to single precision
    // Lattices with more than two slots per lane and colour: the neighbour
    // table with each half index scaled to a byte offset (16 h, the
    // double2 stride; null when 16 half > 65535) and the links once each,
    // U_{i,mu} of the site (c, h) at [c][mu][half]: the backward
    // coefficient of a site is the conjugate of its backward neighbour's
    // forward link.
    const uint4 *nbo;               // [2][half] 8 x u16 byte offsets 16 h (forward mu, then backward)
    const uint4 *nbo32;             // the same scaled for 8-byte sites, 8 h (single-precision kernel)
    const double2 *link64;          // [2][d][half]
    const float2 *link32;           // same, rounded to single precision
};

// Wavefronts per workgroup of the wave kernel; each needs V float2 of
// private scratch for the single-to-double promotion.
constexpr int GC_WAVES = 4;

// Wavefronts (starts) per workgroup of the register-resident kernel used
// above two slots per lane; each start takes 8V bytes of LDS.
constexpr int GC_WAVES_RR = 8;
inline int gc_wave_starts_per_wg(int ns) { return ns > 2 ? GC_WAVES_RR : GC_WAVES; }

// Kernels with more than two slots per lane (ns > 2) stage the links of
// their first gc_links_in_lds(d, ns) directions (both colours, double
// precision, 16 V bytes per direction) in LDS beside the neighbour table and
// the GC_WAVES_RR exchange regions: as many as fit in 160 KiB for the
// largest lattice of the instantiated slot count (half <= 64 ns).
constexpr int gc_links_in_lds(int d, int ns)
{
    const long V = 128L * ns;
    const long room = 160L * 1024 - 16 * V - (long)GC_WAVES_RR * 8 * V;
    const long dl = (ns > 2 && room > 0) ? room / (16 * V) : 0;
    return dl < d ? (int)dl : d;
}

// The single-precision phase of mixed launches above two slots per lane
// runs in its own kernel: GC_WAVES_RR32 starts per workgroup (three
// wavefronts per SIMD), exchange regions of 4V bytes, the links of
// gc_links_in_lds32(d, ns) directions in single precision in LDS (8 bytes
// per site and colour); converged states go to HBM promoted to double
// precision for the double-precision kernel.
constexpr int GC_WAVES_RR32 = 12;
constexpr int gc_links_in_lds32(int d, int ns)
{
    const long V = 128L * ns;
    const long room = 160L * 1024 - 16 * V - (long)GC_WAVES_RR32 * 4 * V;
    const long dl = (ns > 2 && room > 0) ? room / (8 * V) : 0;
    return dl < d ? (int)dl : d;
}
constexpr size_t gc_rr32_links_bytes(int d, int ns) { return (size_t)2 * gc_links_in_lds32(d, ns) * 64 * ns * 8; }
constexpr size_t gc_rr32_lds_bytes(int d, int ns, int V)
{
    return gc_rr32_links_bytes(d, ns) + 16 * (size_t)V + (size_t)GC_WAVES_RR32 * 4 * V;
}

// LDS of the exchange-region kernel for ns (the instantiated slot count) and
// V sites: the staged link planes first (2 d_l planes of 64 ns double2, a
// size fixed at compile time, so that their addresses are immediates), then
// the neighbour table (16V) and one exchange region per start (8V).
constexpr size_t gc_rr_links_bytes(int d, int ns) { return (size_t)2 * gc_links_in_lds(d, ns) * 64 * ns * 16; }
constexpr size_t gc_rr_lds_bytes(int d, int ns, int V)
{
    return gc_rr_links_bytes(d, ns) + 16 * (size_t)V + (size_t)GC_WAVES_RR * 8 * V;
}

// variant = coef_lds | creg << 1 | rm << 3: coefficient table staged in LDS
// (else read from global memory) and the number of colours (0..2) whose
// coefficients a lane keeps in registers (gc_wave_creg_max(d, ns) at most),
// both for ns <= 2; rm, for ns > 2, the relax mode gc_wave_relax_mode(omega,
// stop_norm).
hipError_t gc_wave_occupancy(int d, int ns, int variant, size_t lds, int *per_cu);
hipError_t gc_launch_wave(int d, int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,
                          unsigned long long *job_next, int variant, float2 *bounce, int grid, size_t lds,
                          hipStream_t s);
int gc_wave_creg_max(int d, int ns);
// The single-precision kernel of mixed launches (ns > 2): relax mode rm as
// for gc_launch_wave.
hipError_t gc_wave32_occupancy(int d, int ns, int rm, size_t lds, int *per_cu);
hipError_t gc_launch_wave32(int d, int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,
                            unsigned long long *job_next, int rm, int grid, size_t lds, hipStream_t s);
// Relax mode of the exchange-region kernel: 1 plain relaxation (omega = 1),
// 2 plain relaxation in the single-precision phase only (omega rounds to 1
// in single precision), 0 over-relaxation; plus 4 for the max |div| stopping
// norm (stop_norm != 0).
inline int gc_wave_relax_mode(double omega, int stop_norm)
{
    return (omega == 1.0 ? 1 : (float)omega == 1.0f ? 2 : 0) | (stop_norm ? 4 : 0);
}
// Added to a relax mode (0..6) of gc_launch_wave's variant where every orbit
// of the launch fills all slots of a lane but the last (ceil(half / 64)
// equals the instantiated slot count): the double-precision kernel then
// tests the last slot only.  Not for the single-precision kernel.
constexpr int GC_RM_FULL_SLOTS = 8;

// Workgroup-per-start variant (lattices with more than 128 slots per
// colour): wps wavefronts share a start, at most two slots per thread.
// gc_wps_for(ns) gives wps for ns slots per lane of the one-wavefront layout
// (0 when that layout is used, -1 when too large).  LDS: 32V bytes.
int gc_wps_for(int ns);
hipError_t gc_wps_occupancy(int d, int wps, size_t lds, int *per_cu);
hipError_t gc_launch_wps(int d, int wps, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,
                         unsigned long long *job_next, float2 *bounce, int grid, size_t lds, hipStream_t s);
