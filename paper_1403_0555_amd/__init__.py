"""MI355X (gfx950) Gribov-copy enumerator for compact U(1) lattice gauge fields.

The work runs in ``libgribov.so`` (hand-written HIP kernels behind the C ABI
declared in ``include/gribov.h``).  This package is the thin ctypes binding:
same entry-point names, argument marshalling only.  Importing it does not
need a GPU; creating a context does.
"""
from ._capi import (  # noqa: F401
    GC_OK, GC_EINVAL, GC_ENOMEM, GC_EUNSUPPORTED, GC_EDEVICE, GC_EBUSY, GC_ETIMEOUT, GC_ENOTFOUND, GC_ESTATE,
    GC_FP64, GC_MIXED, GC_MEAN_SQ, GC_MAX_ABS,
    GC_START_PENDING, GC_START_CONVERGED, GC_START_NONCONVERGED, GC_START_BADNUM,
    GC_FLAG_IN_REGION, GC_FLAG_SINGULAR, GC_FLAG_SADDLE, GC_FLAG_COLLISION, GC_FLAG_LANCZOS_CAP,
    GC_ORBIT_IDLE, GC_ORBIT_QUEUED, GC_ORBIT_RUNNING, GC_ORBIT_DONE, GC_ORBIT_ERROR,
    GC_HIST_X, GC_HIST_REL, GC_HIST_COPIES, GC_HIST_STARTS,
    GcError, COPY_DTYPE, START_DTYPE, EXPORTED_SYMBOLS,
    lib, lib_path, gc_version, gc_status_str, gc_lattice_check, gc_solve_params_default,
    Context, SolveParams,
)
