"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point declared in include/gribov.h,
and validate arguments on the host before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1403_0555_amd as gc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gribov.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:gc_status|const char \*)\s*(gc_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_binding_names():
    assert _declared() == sorted(gc.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = gc.lib()
    for name in _declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", gc.lib_path()], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(gc_\w+)", out))
    assert set(_declared()) <= exported


def test_library_is_gfx950_hip():
    # the shared object carries a gfx950 code object
    data = open(gc.lib_path(), "rb").read()
    assert b"gfx950" in data


def test_version_and_status_text():
    assert re.match(r"\d+\.\d+\.\d+$", gc.gc_version())
    assert gc.gc_status_str(gc.GC_OK) == "ok"
    assert "budget" in gc.gc_status_str(gc.GC_ENOMEM)
    assert gc.gc_status_str(12345) == "unknown status"


@pytest.mark.parametrize("extent,status,K", [
    ((4, 4), 0, 2), ((3, 3), 0, 3), ((5, 5), 0, 5), ((2,), 0, 2), ((7,), 0, 7), ((6, 6, 6, 6), 0, 2),
    ((8, 8, 8, 8), 0, 2), ((3, 5), gc.GC_EUNSUPPORTED, 0), ((1, 4), gc.GC_EINVAL, 0), ((), gc.GC_EINVAL, 0),
    ((2, 2, 2, 2, 2), gc.GC_EINVAL, 0), ((10, 10, 10, 10), gc.GC_EUNSUPPORTED, 0)])
def test_lattice_check(extent, status, K):
    st, k = gc.gc_lattice_check(extent)
    assert st == status
    if status == 0:
        assert k == K


def test_default_params():
    p = gc.gc_solve_params_default()
    assert p.omega == 1.0 and p.eps32 == 1e-6 and p.eps64 == 1e-14 and p.lambda_tol == 1e-6
    assert p.precision == gc.GC_FP64 and p.stop_norm == gc.GC_MEAN_SQ and p.check_every == 1
    assert p.max_sweeps == 100000 and p.lanczos_max_iter == 300


def test_null_arguments_rejected_without_device():
    L = gc.lib()
    assert L.gc_create(None, None) == gc.GC_EINVAL
    assert L.gc_destroy(None) == gc.GC_EINVAL
    assert L.gc_solve_params_default(None) == gc.GC_EINVAL
    assert L.gc_lattice_check(None, None) == gc.GC_EINVAL
    assert L.gc_launch(None, 1, 10, None) == gc.GC_EINVAL
    assert L.gc_poll(None, 1, None) == gc.GC_EINVAL
    sizes = (ctypes.c_uint64 * 2)(4, 2)
    out = (ctypes.c_uint64 * 2)()
    # bad counts, missing arrays and decreasing sizes fail before any device call
    assert L.gc_paper_saturation(None, 1, -1, None, None) == gc.GC_EINVAL
    assert L.gc_paper_saturation(None, 1, 2, None, out) == gc.GC_EINVAL
    assert L.gc_paper_saturation(None, 1, 2, sizes, out) == gc.GC_EINVAL
    assert L.gc_saturation(None, 1, 2, sizes, 0, None) == gc.GC_EINVAL


def test_no_device_is_reported(monkeypatch):
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert gc.lib().gc_create(None, ctypes.byref(h)) == gc.GC_EDEVICE


def test_su2_reduction_arguments_checked_without_device():
    """gc_orbit_load_su2 validates the lattice, the links and the parameters
    before it touches the context or the device."""
    from paper_1403_0555_amd._capi import gc_lattice, gc_mag_params, gc_mag_info
    import gribov_inputs as GI
    L = gc.lib()
    P = ctypes.POINTER(ctypes.c_double)
    out, info = ctypes.c_uint64(), gc_mag_info()

    def call(extent, links, eps=1e-20, max_sweeps=100000):
        lat = gc_lattice(len(extent), (ctypes.c_int32 * 4)(*(list(extent) + [1] * (4 - len(extent)))), 0)
        prm = gc_mag_params(eps, max_sweeps)
        ptr = links.ctypes.data_as(P) if links is not None else None
        return L.gc_orbit_load_su2(None, ctypes.byref(lat), ptr, 0, ctypes.byref(prm), ctypes.byref(info),
                                   ctypes.byref(out))

    good = np.ascontiguousarray(GI.su2_links((4, 4), 0, 0))
    assert call((4, 4), None) == gc.GC_EINVAL
    assert call((6, 3), np.ascontiguousarray(GI.su2_links((6, 3), 0, 0))) == gc.GC_EUNSUPPORTED
    assert call((10, 10, 10, 10), np.zeros((4, 10000, 4))) == gc.GC_EUNSUPPORTED
    bad = good.copy()
    bad[0, 5, 1] += 1e-6
    assert call((4, 4), bad) == gc.GC_EINVAL
    assert call((4, 4), good, max_sweeps=0) == gc.GC_EINVAL
    assert call((4, 4), good, max_sweeps=10**6 + 1) == gc.GC_EINVAL
    assert call((4, 4), good, eps=float("nan")) == gc.GC_EINVAL
    # valid arguments: the missing context is the only fault left
    assert call((4, 4), good) == gc.GC_EINVAL
