// Wavefront-per-start and workgroup-per-start relax kernels of 1-dimensional
// lattices (see gc_wave_kern.h); one translation unit per dimension.
#include "gc_wave_kern.h"

#define GC_NS_LIST_D1(FN, D, ...) return ns <= 1 ? FN<1, 1, 4>(__VA_ARGS__) : ns <= 4 ? FN<1, 4, 4>(__VA_ARGS__) : ns <= 12 ? FN<1, 12, 4>(__VA_ARGS__) : FN<1, 16, 4>(__VA_ARGS__);

GC_WAVE_DEFINE_DIM(1, GC_NS_LIST_D1)
