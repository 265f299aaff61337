// Colour-split tables and launch entry points of the wavefront-per-start
// solver (lattices whose extents are all even).
#pragma once

#include "gc_internal.h"

struct GcWaveOrbit {
    int32_t half, pad;              // V / 2
    const uint16_t *loc;            // [V] site -> c * half + h
    const uint4 *nb;                // [2][half] neighbour half indices, 8 x u16 (forward mu, then backward)
    const uint32_t *desc;           // [2][half] site i | forward-wrap bits << 12 | backward-wrap bits << 16
    const double2 *coef64;          // [2][2d][half] U_{i,k} (forward) / conj(U_{i-k,k}) (backward)
    const float2 *coef32;           // same, rounded to single precision
};

// Wavefronts per workgroup of the wave kernel; each needs V float2 of
// private scratch for the single-to-double promotion.
constexpr int GC_WAVES = 4;

// variant = coef_lds | creg << 1: coefficient table staged in LDS (else
// read from global memory) and the number of colours (0..2) whose
// coefficients a lane keeps in registers (gc_wave_creg_max(d, ns) at most).
hipError_t gc_wave_occupancy(int d, int ns, int variant, size_t lds, int *per_cu);
hipError_t gc_launch_wave(int d, int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,
                          unsigned long long *job_next, int variant, float2 *bounce, int grid, size_t lds,
                          hipStream_t s);
int gc_wave_creg_max(int d, int ns);

// Workgroup-per-start variant (lattices with more than 128 slots per
// colour): wps wavefronts share a start, at most two slots per thread.
// gc_wps_for(ns) gives wps for ns slots per lane of the one-wavefront layout
// (0 when that layout is used, -1 when too large).  LDS: 32V bytes.
int gc_wps_for(int ns);
hipError_t gc_wps_occupancy(int d, int wps, size_t lds, int *per_cu);
hipError_t gc_launch_wps(int d, int wps, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,
                         unsigned long long *job_next, float2 *bounce, int grid, size_t lds, hipStream_t s);
