// Wavefront-per-start and workgroup-per-start relax kernels of 2-dimensional
// lattices (see gc_wave_kern.h); one translation unit per dimension.
#include "gc_wave_kern.h"

#define GC_NS_LIST_D2(FN, D, ...) return ns <= 1 ? FN<2, 1, 4>(__VA_ARGS__) : ns <= 2 ? FN<2, 2, 4>(__VA_ARGS__) : ns <= 4 ? FN<2, 4, 4>(__VA_ARGS__) : ns <= 12 ? FN<2, 12, 4>(__VA_ARGS__) : FN<2, 16, 4>(__VA_ARGS__);

GC_WAVE_DEFINE_DIM(2, GC_NS_LIST_D2)
