// Line-segment Lanczos filter kernels of 1-dimensional lattices (see
// gc_lanczos_kern.h); one translation unit per dimension.
#include "gc_lanczos_kern.h"

GC_LANCZOS_DEFINE_DIM(1)
