// Wavefront-per-start and workgroup-per-start relax kernels of 4-dimensional
// lattices (see gc_wave_kern.h); one translation unit per dimension.
#include "gc_wave_kern.h"

#define GC_NS_LIST_D4(FN, D, ...) return ns <= 1 ? FN<4, 1, 4>(__VA_ARGS__) : ns <= 2 ? FN<4, 2, 4>(__VA_ARGS__) : ns <= 4 ? FN<4, 4, 4>(__VA_ARGS__) : ns <= 11 ? FN<4, 11, 4>(__VA_ARGS__) : FN<4, 16, 4>(__VA_ARGS__);

GC_WAVE_DEFINE_DIM(4, GC_NS_LIST_D4)
