// Wavefront-per-start and workgroup-per-start relax kernels of 3-dimensional
// lattices (see gc_wave_kern.h); one translation unit per dimension.
#include "gc_wave_kern.h"

#define GC_NS_LIST_D3(FN, D, ...) return ns <= 2 ? FN<3, 2, 4>(__VA_ARGS__) : ns <= 4 ? FN<3, 4, 4>(__VA_ARGS__) : ns <= 8 ? FN<3, 8, 4>(__VA_ARGS__) : FN<3, 16, 4>(__VA_ARGS__);

GC_WAVE_DEFINE_DIM(3, GC_NS_LIST_D3)
