// Dispatch of the two-colour relax kernels by lattice dimension (the kernels
// themselves are in gc_wave_kern.h, instantiated per dimension in
// gc_wave1.hip .. gc_wave4.hip).
#include "gc_wave.h"

#define GC_WAVE_DECLARE_DIM(D)                                                                              \
    hipError_t gc_wave_occupancy_d##D(int ns, int variant, size_t lds, int *per_cu);                         \
    hipError_t gc_launch_wave_d##D(int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,      \
                                   unsigned long long *job_next, int variant, float2 *bounce, int grid,      \
                                   size_t lds, hipStream_t s);                                               \
    hipError_t gc_wps_occupancy_d##D(int wps, size_t lds, int *per_cu);                                      \
    hipError_t gc_launch_wps_d##D(int wps, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,      \
                                  unsigned long long *job_next, float2 *bounce, int grid, size_t lds,        \
                                  hipStream_t s);
#define GC_WAVE32_DECLARE_DIM(D)                                                                            \
    hipError_t gc_wave32_occupancy_d##D(int ns, int rm, size_t lds, int *per_cu);                            \
    hipError_t gc_launch_wave32_d##D(int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,    \
                                     unsigned long long *job_next, int rm, int grid, size_t lds, hipStream_t s);
GC_WAVE32_DECLARE_DIM(1)
GC_WAVE32_DECLARE_DIM(2)
GC_WAVE32_DECLARE_DIM(3)
GC_WAVE32_DECLARE_DIM(4)
GC_WAVE_DECLARE_DIM(1)
GC_WAVE_DECLARE_DIM(2)
GC_WAVE_DECLARE_DIM(3)
GC_WAVE_DECLARE_DIM(4)

hipError_t gc_wave_occupancy(int d, int ns, int variant, size_t lds, int *per_cu)
{
    switch (d) {
    case 1: return gc_wave_occupancy_d1(ns, variant, lds, per_cu);
    case 2: return gc_wave_occupancy_d2(ns, variant, lds, per_cu);
    case 3: return gc_wave_occupancy_d3(ns, variant, lds, per_cu);
    case 4: return gc_wave_occupancy_d4(ns, variant, lds, per_cu);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gc_launch_wave(int d, int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,
                          unsigned long long *job_next, int variant, float2 *bounce, int grid, size_t lds,
                          hipStream_t s)
{
    switch (d) {
    case 1: return gc_launch_wave_d1(ns, jobs, worbs, n_jobs, job_next, variant, bounce, grid, lds, s);
    case 2: return gc_launch_wave_d2(ns, jobs, worbs, n_jobs, job_next, variant, bounce, grid, lds, s);
    case 3: return gc_launch_wave_d3(ns, jobs, worbs, n_jobs, job_next, variant, bounce, grid, lds, s);
    case 4: return gc_launch_wave_d4(ns, jobs, worbs, n_jobs, job_next, variant, bounce, grid, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gc_wave32_occupancy(int d, int ns, int rm, size_t lds, int *per_cu)
{
    switch (d) {
    case 1: return gc_wave32_occupancy_d1(ns, rm, lds, per_cu);
    case 2: return gc_wave32_occupancy_d2(ns, rm, lds, per_cu);
    case 3: return gc_wave32_occupancy_d3(ns, rm, lds, per_cu);
    case 4: return gc_wave32_occupancy_d4(ns, rm, lds, per_cu);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gc_launch_wave32(int d, int ns, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,
                            unsigned long long *job_next, int rm, int grid, size_t lds, hipStream_t s)
{
    switch (d) {
    case 1: return gc_launch_wave32_d1(ns, jobs, worbs, n_jobs, job_next, rm, grid, lds, s);
    case 2: return gc_launch_wave32_d2(ns, jobs, worbs, n_jobs, job_next, rm, grid, lds, s);
    case 3: return gc_launch_wave32_d3(ns, jobs, worbs, n_jobs, job_next, rm, grid, lds, s);
    case 4: return gc_launch_wave32_d4(ns, jobs, worbs, n_jobs, job_next, rm, grid, lds, s);
    default: return hipErrorInvalidValue;
    }
}

// Register-held coefficients are instantiated where a lane's slots are few
// (at most two per colour): creg 1 holds colour 0, creg 2 both colours.
int gc_wave_creg_max(int d, int ns)
{
    (void)d;
    return ns <= 2 ? 2 : 0;
}

// Wavefronts per start of the workgroup-per-start variant for a lattice with
// ns slots per lane in the one-wavefront layout (0: use that layout).
int gc_wps_for(int ns)
{
    if (ns <= 2) return 0;
    static const int w[] = {2, 4, 6, 8, 16};
    for (int x : w)
        if (2 * x >= ns) return x;
    return -1;
}

hipError_t gc_wps_occupancy(int d, int wps, size_t lds, int *per_cu)
{
    switch (d) {
    case 1: return gc_wps_occupancy_d1(wps, lds, per_cu);
    case 2: return gc_wps_occupancy_d2(wps, lds, per_cu);
    case 3: return gc_wps_occupancy_d3(wps, lds, per_cu);
    case 4: return gc_wps_occupancy_d4(wps, lds, per_cu);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gc_launch_wps(int d, int wps, const GcJobDev *jobs, const GcWaveOrbit *worbs, int n_jobs,
                         unsigned long long *job_next, float2 *bounce, int grid, size_t lds, hipStream_t s)
{
    switch (d) {
    case 1: return gc_launch_wps_d1(wps, jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);
    case 2: return gc_launch_wps_d2(wps, jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);
    case 3: return gc_launch_wps_d3(wps, jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);
    case 4: return gc_launch_wps_d4(wps, jobs, worbs, n_jobs, job_next, bounce, grid, lds, s);
    default: return hipErrorInvalidValue;
    }
}
