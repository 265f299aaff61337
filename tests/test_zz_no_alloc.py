"""GPU: the allocation-free entry point against gc_launch.

gc_launch_static runs the path of gc_launch for one orbit in a static device
array, writing to caller-owned device buffers.  Two calls in a row (the
second with a smaller input, so the array holds the first call's leftovers)
must reproduce gc_launch's copies exactly, and charge nothing to the
context."""
import ctypes

import numpy as np
import pytest

import gribov_inputs as GI
import paper_1403_0555_amd as gc

pytestmark = pytest.mark.gpu


def _hip():
    gc.lib()
    return ctypes.CDLL("libamdhip64.so.7")


def _sorted(c):
    return c[np.lexsort((c["key_lo"], c["key_hi"]))]


def test_static_launch_equals_gc_launch():
    hip = _hip()
    cases = [((4, 4, 4, 4), 3000, gc.SolveParams(omega=1.0), 0),
             ((6, 6), 500, gc.SolveParams(omega=1.7, precision="mixed"), 3)]
    cap = 100_000          # copies buffer: room for the refused call below too
    stream = ctypes.c_void_p()
    copies_dev, n_dev, cnt_dev = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipStreamCreateWithFlags(ctypes.byref(stream), 1) == 0
    assert hip.hipMalloc(ctypes.byref(copies_dev), ctypes.c_size_t(cap * gc.COPY_DTYPE.itemsize)) == 0
    assert hip.hipMalloc(ctypes.byref(n_dev), ctypes.c_size_t(8)) == 0
    assert hip.hipMalloc(ctypes.byref(cnt_dev), ctypes.c_size_t(64)) == 0
    try:
        with gc.Context(0) as ctx:
            for ext, n, p, oi in cases:
                h = ctx.gc_orbit_load(ext, GI.orbit_angles(ext, 0, oi), oi)
                ctx.gc_launch(h, n, p)
                assert ctx.gc_wait(h) == gc.GC_OK
                ref, prog = ctx.gc_fetch(h), ctx.gc_poll(h)
                before = ctx.gc_memory_info()
                ctx.gc_launch_static(h, n, p, stream.value, copies_dev.value, cap, n_dev.value, cnt_dev.value)
                assert hip.hipStreamSynchronize(stream) == 0
                m = ctypes.c_uint64()
                assert hip.hipMemcpy(ctypes.byref(m), n_dev, ctypes.c_size_t(8), 2) == 0
                got = np.zeros(m.value, dtype=gc.COPY_DTYPE)
                assert hip.hipMemcpy(got.ctypes.data_as(ctypes.c_void_p), copies_dev,
                                     ctypes.c_size_t(m.value * gc.COPY_DTYPE.itemsize), 2) == 0
                cnt = np.zeros(8, dtype=np.uint64)
                assert hip.hipMemcpy(cnt.ctypes.data_as(ctypes.c_void_p), cnt_dev, ctypes.c_size_t(64), 2) == 0
                got = _sorted(got)
                assert len(got) == len(ref) == prog["distinct"]
                for f in ref.dtype.names:
                    assert np.array_equal(got[f], ref[f], equal_nan=ref[f].dtype.kind == "f"), f
                assert int(cnt[0]) == n and int(cnt[1]) == prog["converged"] and int(cnt[3]) == len(ref)
                assert int(cnt[4]) == prog["sweeps_total"] and int(cnt[6]) == 0
                assert ctx.gc_memory_info() == before
                # the orbit's own results are untouched
                assert np.array_equal(ctx.gc_fetch(h)["key_hi"], ref["key_hi"])
            # beyond the static array: refused with a clear error
            big = ctx.gc_orbit_load((4, 4, 4, 4), GI.orbit_angles((4, 4, 4, 4), 0, 0), 0)
            with pytest.raises(gc.GcError) as e:
                ctx.gc_launch_static(big, 100_000, None, stream.value, copies_dev.value, cap, n_dev.value)
            assert e.value.status == gc.GC_ENOMEM
            assert "static array" in ctx.gc_last_error()
            # a copies buffer smaller than the start count is refused too
            with pytest.raises(gc.GcError) as e2:
                ctx.gc_launch_static(big, 10, None, stream.value, copies_dev.value, 5, n_dev.value)
            assert e2.value.status == gc.GC_EINVAL
    finally:
        hip.hipFree(copies_dev)
        hip.hipFree(n_dev)
        hip.hipFree(cnt_dev)
        hip.hipStreamDestroy(stream)
