"""ctypes binding of include/gribov.h (argument marshalling only).

Every computation happens in libgribov.so on the GPU.  If the library is not
built, ``lib()`` raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libgribov.so")

GC_OK, GC_EINVAL, GC_ENOMEM, GC_EUNSUPPORTED, GC_EDEVICE = 0, -1, -2, -3, -4
GC_EBUSY, GC_ETIMEOUT, GC_ENOTFOUND, GC_ESTATE = -5, -6, -7, -8
GC_FP64, GC_MIXED = 0, 1
GC_MEAN_SQ, GC_MAX_ABS = 0, 1
GC_START_PENDING, GC_START_CONVERGED, GC_START_NONCONVERGED, GC_START_BADNUM = 0, 1, 2, 3
GC_FLAG_IN_REGION, GC_FLAG_SINGULAR, GC_FLAG_SADDLE, GC_FLAG_COLLISION, GC_FLAG_LANCZOS_CAP = 1, 2, 4, 8, 16
GC_ORBIT_IDLE, GC_ORBIT_QUEUED, GC_ORBIT_RUNNING, GC_ORBIT_DONE, GC_ORBIT_ERROR = 0, 1, 2, 3, 4
GC_HIST_X, GC_HIST_REL = 0, 1
GC_HIST_COPIES, GC_HIST_STARTS = 0, 1

EXPORTED_SYMBOLS = [
    "gc_version", "gc_status_str", "gc_lattice_check", "gc_solve_params_default",
    "gc_create", "gc_destroy", "gc_orbit_load", "gc_orbit_random", "gc_orbit_angles",
    "gc_launch", "gc_launch_batch", "gc_poll", "gc_wait", "gc_fetch", "gc_fetch_starts",
    "gc_fetch_state", "gc_fetch_start_state", "gc_release", "gc_last_error", "gc_kernel_time_ms", "gc_launch_bytes",
    "gc_memory_info", "gc_autotune", "gc_saturation", "gc_paper_saturation", "gc_launch_static",
    "gc_launch_from", "gc_histogram", "gc_orbit_load_su2",
]


class gc_tune_result(ctypes.Structure):
    _fields_ = [("relax_variant", ctypes.c_int32), ("post_block", ctypes.c_int32),
                ("post_sites_per_thread", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("relax_ms", ctypes.c_double), ("post_ms", ctypes.c_double)]


class gc_mag_params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("max_sweeps", ctypes.c_uint64)]


class gc_mag_info(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_uint64), ("R", ctypes.c_double), ("converged", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class gc_ctx_params(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_streams", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("hip_stream", ctypes.c_void_p), ("tune_cache", ctypes.c_char_p)]


class gc_lattice(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("extent", ctypes.c_int32 * 4), ("antiperiodic", ctypes.c_uint32)]


class gc_solve_params(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("eps32", ctypes.c_double), ("eps64", ctypes.c_double),
                ("lambda_tol", ctypes.c_double), ("precision", ctypes.c_int32), ("stop_norm", ctypes.c_int32),
                ("check_every", ctypes.c_uint32), ("lanczos_max_iter", ctypes.c_uint32),
                ("max_sweeps", ctypes.c_uint64), ("start_seed", ctypes.c_uint64), ("first_start", ctypes.c_uint64),
                ("sync_batch", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class gc_progress(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("pad", ctypes.c_int32)] + [
        (n, ctypes.c_uint64) for n in ("n_starts", "starts_done", "converged", "nonconverged", "distinct",
                                       "in_region", "saddles", "singular", "collisions", "sweeps_total",
                                       "site_updates", "lanczos_runs", "paper_count")] + [
        ("submit_to_done_ms", ctypes.c_double), ("device_ms", ctypes.c_double), ("post_ms", ctypes.c_double),
        ("filter_ms", ctypes.c_double), ("in_region_hits", ctypes.c_uint64), ("lanczos_iters", ctypes.c_uint64)]


COPY_DTYPE = np.dtype([("key_hi", np.uint64), ("key_lo", np.uint64), ("F", np.float64), ("x", np.float64),
                       ("lambda2", np.float64), ("hits", np.uint64), ("first_start", np.uint64),
                       ("rep_start", np.uint64), ("flags", np.uint32), ("lanczos_iters", np.uint32)])
START_DTYPE = np.dtype([("status", np.int32), ("sweeps32", np.uint32), ("sweeps64", np.uint32),
                        ("lanczos_iters", np.uint32), ("F", np.float64), ("D", np.float64),
                        ("lambda2", np.float64), ("key_hi", np.uint64), ("key_lo", np.uint64),
                        ("paper_X", np.uint32), ("flags", np.uint32)])
assert COPY_DTYPE.itemsize == 72 and START_DTYPE.itemsize == 64


class GcError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = "%s failed: %s (%d)" % (where, gc_status_str(status), status)
        if detail:
            msg += ": " + detail
        super().__init__(msg)


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libgribov.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError("libgribov.so is not built; run `python -m paper_1403_0555_amd.build`")
    L = ctypes.CDLL(_LIB_PATH)
    P, vp = ctypes.POINTER, ctypes.c_void_p
    u64, i32, i64 = ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
    sig = {
        "gc_version": ([], ctypes.c_char_p),
        "gc_status_str": ([i32], ctypes.c_char_p),
        "gc_lattice_check": ([P(gc_lattice), P(i32)], i32),
        "gc_solve_params_default": ([P(gc_solve_params)], i32),
        "gc_create": ([P(gc_ctx_params), P(vp)], i32),
        "gc_destroy": ([vp], i32),
        "gc_orbit_load": ([vp, P(gc_lattice), P(ctypes.c_double), u64, P(u64)], i32),
        "gc_orbit_random": ([vp, P(gc_lattice), u64, u64, P(u64)], i32),
        "gc_orbit_load_su2": ([vp, P(gc_lattice), P(ctypes.c_double), u64, P(gc_mag_params), P(gc_mag_info),
                               P(u64)], i32),
        "gc_orbit_angles": ([vp, u64, P(ctypes.c_double)], i32),
        "gc_launch": ([vp, u64, u64, P(gc_solve_params)], i32),
        "gc_launch_batch": ([vp, i32, P(u64), P(u64), P(gc_solve_params)], i32),
        "gc_poll": ([vp, u64, P(gc_progress)], i32),
        "gc_wait": ([vp, u64, i64], i32),
        "gc_fetch": ([vp, u64, u64, u64, vp, P(u64), P(u64)], i32),
        "gc_fetch_starts": ([vp, u64, u64, u64, vp, P(u64)], i32),
        "gc_fetch_state": ([vp, u64, u64, u64, P(ctypes.c_double)], i32),
        "gc_fetch_start_state": ([vp, u64, u64, P(ctypes.c_double)], i32),
        "gc_release": ([vp, u64], i32),
        "gc_last_error": ([vp, ctypes.c_char_p, ctypes.c_size_t], i32),
        "gc_kernel_time_ms": ([vp, u64, P(ctypes.c_double)], i32),
        "gc_launch_bytes": ([vp, u64, u64, P(gc_solve_params), P(u64)], i32),
        "gc_memory_info": ([vp, P(u64), P(u64), P(u64)], i32),
        "gc_autotune": ([vp, u64, u64, P(gc_solve_params), P(gc_tune_result)], i32),
        "gc_saturation": ([vp, u64, i32, P(u64), i32, P(u64)], i32),
        "gc_paper_saturation": ([vp, u64, i32, P(u64), P(u64)], i32),
        "gc_launch_static": ([vp, u64, u64, P(gc_solve_params), vp, vp, u64, vp, vp], i32),
        "gc_launch_from": ([vp, u64, u64, P(ctypes.c_double), P(gc_solve_params)], i32),
        "gc_histogram": ([vp, i32, P(u64), i32, i32, ctypes.c_uint32, ctypes.c_double, ctypes.c_double, i32,
                          P(u64)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def gc_version() -> str:
    return lib().gc_version().decode()


def gc_status_str(s: int) -> str:
    return lib().gc_status_str(int(s)).decode()


def _lattice(extent, antiperiodic: int = 0) -> gc_lattice:
    ext = [int(n) for n in extent]
    lat = gc_lattice()
    lat.dim = len(ext)
    for k in range(4):
        lat.extent[k] = ext[k] if k < len(ext) else 0
    lat.antiperiodic = int(antiperiodic)
    return lat


def gc_lattice_check(extent, antiperiodic: int = 0):
    """Returns (status, n_colours)."""
    K = ctypes.c_int32(0)
    lat = _lattice(extent, antiperiodic)
    st = lib().gc_lattice_check(ctypes.byref(lat), ctypes.byref(K))
    return int(st), int(K.value)


def gc_solve_params_default() -> gc_solve_params:
    p = gc_solve_params()
    lib().gc_solve_params_default(ctypes.byref(p))
    return p


@dataclass
class SolveParams:
    omega: float = 1.0
    precision: str = "fp64"       # "fp64" | "mixed"
    eps32: float = 1e-6
    eps64: float = 1e-14
    lambda_tol: float = 1e-6
    stop_norm: str = "mean_sq"    # "mean_sq" | "max_abs"
    check_every: int = 1
    lanczos_max_iter: int = 300
    max_sweeps: int = 100_000
    start_seed: int = 0
    first_start: int = 0
    sync_batch: int = 0           # > 0: batch-synchronous stop over batches of this many starts

    def c(self) -> gc_solve_params:
        p = gc_solve_params()
        p.omega, p.eps32, p.eps64, p.lambda_tol = self.omega, self.eps32, self.eps64, self.lambda_tol
        p.precision = GC_MIXED if self.precision == "mixed" else GC_FP64
        p.stop_norm = GC_MAX_ABS if self.stop_norm == "max_abs" else GC_MEAN_SQ
        p.check_every = self.check_every
        p.lanczos_max_iter = self.lanczos_max_iter
        p.max_sweeps, p.start_seed, p.first_start = self.max_sweeps, self.start_seed, self.first_start
        p.sync_batch = self.sync_batch
        return p


class Context:
    """One gc_ctx.  Methods mirror the C entry points."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, n_streams: int = 0, hip_stream: int = 0,
                 tune_cache: str | None = None):
        self._L = lib()
        self._tune_cache = tune_cache.encode() if tune_cache else None
        prm = gc_ctx_params(device, n_streams, hbm_budget_bytes, hip_stream or None, self._tune_cache)
        h = ctypes.c_void_p()
        st = self._L.gc_create(ctypes.byref(prm), ctypes.byref(h))
        if st != GC_OK:
            raise GcError(st, "gc_create")
        self._h = h
        self.extent = {}

    # -- helpers -----------------------------------------------------------
    def _check(self, st, where):
        if st != GC_OK:
            buf = ctypes.create_string_buffer(512)
            self._L.gc_last_error(self._h, buf, 512)
            raise GcError(st, where, buf.value.decode(errors="replace"))

    def close(self):
        if getattr(self, "_h", None):
            self._L.gc_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- orbits --------------------------------------------------------------
    def gc_orbit_load(self, extent, phi, orbit_index: int = 0, antiperiodic: int = 0) -> int:
        lat = _lattice(extent, antiperiodic)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        out = ctypes.c_uint64()
        st = self._L.gc_orbit_load(self._h, ctypes.byref(lat), phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   orbit_index, ctypes.byref(out))
        self._check(st, "gc_orbit_load")
        self.extent[out.value] = tuple(int(n) for n in extent)
        return out.value

    def gc_orbit_load_su2(self, extent, links, orbit_index: int = 0, eps: float = 1e-20,
                          max_sweeps: int = 100000):
        """SU(2) links [dim][V][4] (unit quaternions) through the maximal
        Abelian reduction; returns (orbit handle, {sweeps, R, converged})."""
        lat = _lattice(extent, 0)
        links = np.ascontiguousarray(links, dtype=np.float64)
        d, V = len(extent), int(np.prod(extent))
        if links.size != 4 * d * V:
            raise ValueError("links must hold dim x V quaternions")
        prm = gc_mag_params(eps, max_sweeps)
        info = gc_mag_info()
        out = ctypes.c_uint64()
        st = self._L.gc_orbit_load_su2(self._h, ctypes.byref(lat), links.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       orbit_index, ctypes.byref(prm), ctypes.byref(info), ctypes.byref(out))
        self._check(st, "gc_orbit_load_su2")
        self.extent[out.value] = tuple(int(n) for n in extent)
        return out.value, {"sweeps": int(info.sweeps), "R": float(info.R), "converged": bool(info.converged)}

    def gc_orbit_random(self, extent, seed: int = 0, orbit_index: int = 0, antiperiodic: int = 0) -> int:
        lat = _lattice(extent, antiperiodic)
        out = ctypes.c_uint64()
        self._check(self._L.gc_orbit_random(self._h, ctypes.byref(lat), seed, orbit_index, ctypes.byref(out)),
                    "gc_orbit_random")
        self.extent[out.value] = tuple(int(n) for n in extent)
        return out.value

    def gc_orbit_angles(self, orbit: int) -> np.ndarray:
        ext = self.extent[orbit]
        out = np.empty((len(ext), int(np.prod(ext))), dtype=np.float64)
        self._check(self._L.gc_orbit_angles(self._h, orbit, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "gc_orbit_angles")
        return out

    # -- launches ------------------------------------------------------------
    def gc_launch(self, orbit: int, n_starts: int, params: SolveParams | None = None):
        p = (params or SolveParams()).c()
        self._check(self._L.gc_launch(self._h, orbit, n_starts, ctypes.byref(p)), "gc_launch")

    def gc_launch_from(self, orbit: int, theta, params: SolveParams | None = None):
        """Launch from the caller's start angles theta [n_starts][V] (float64)."""
        p = (params or SolveParams()).c()
        t = np.ascontiguousarray(theta, dtype=np.float64)
        if t.ndim != 2:
            raise ValueError("theta must be [n_starts][V]")
        self._check(self._L.gc_launch_from(self._h, orbit, t.shape[0],
                                           t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(p)),
                    "gc_launch_from")

    def gc_histogram(self, orbits, lo: float, hi: float, n_bins: int, quantity: int = GC_HIST_X,
                     weight: int = GC_HIST_COPIES, require_flags: int = 0) -> np.ndarray:
        """Per-orbit counts [n_orbits][n_bins + 2]: underflow, bins, overflow."""
        n = len(orbits)
        o = (ctypes.c_uint64 * n)(*orbits)
        out = np.zeros((n, n_bins + 2), dtype=np.uint64)
        self._check(self._L.gc_histogram(self._h, n, o, quantity, weight, require_flags, lo, hi, n_bins,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), "gc_histogram")
        return out

    def gc_launch_batch(self, orbits, n_starts, params: SolveParams | None = None):
        p = (params or SolveParams()).c()
        n = len(orbits)
        o = (ctypes.c_uint64 * n)(*orbits)
        s = (ctypes.c_uint64 * n)(*n_starts)
        self._check(self._L.gc_launch_batch(self._h, n, o, s, ctypes.byref(p)), "gc_launch_batch")

    def gc_poll(self, orbit: int) -> dict:
        p = gc_progress()
        self._check(self._L.gc_poll(self._h, orbit, ctypes.byref(p)), "gc_poll")
        return {k: getattr(p, k) for k, _ in gc_progress._fields_ if k != "pad"}

    def gc_wait(self, orbit: int, timeout_ms: int = -1) -> int:
        st = self._L.gc_wait(self._h, orbit, timeout_ms)
        if st not in (GC_OK, GC_ETIMEOUT):
            self._check(st, "gc_wait")
        return int(st)

    def gc_fetch(self, orbit: int, out: np.ndarray | None = None) -> np.ndarray:
        """The copy table, ascending by key.  out: a caller-owned contiguous
        COPY_DTYPE array to write into instead of a new one (a caller that
        fetches every launch keeps one); the result is then its first
        n_total records.  ValueError if out cannot hold the table."""
        total = ctypes.c_uint64()
        nw = ctypes.c_uint64()
        if out is not None:
            if out.dtype != COPY_DTYPE or out.ndim != 1 or not out.flags.c_contiguous or not out.flags.writeable:
                raise ValueError("out: a writeable contiguous one-dimensional COPY_DTYPE array")
            self._check(self._L.gc_fetch(self._h, orbit, 0, len(out), out.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(nw), ctypes.byref(total)), "gc_fetch")
            if total.value > len(out):
                raise ValueError("out holds %d records, the table %d" % (len(out), total.value))
            return out[:nw.value]
        self._check(self._L.gc_fetch(self._h, orbit, 0, 0, None, ctypes.byref(nw), ctypes.byref(total)), "gc_fetch")
        out = np.zeros(total.value, dtype=COPY_DTYPE)
        if total.value:
            self._check(self._L.gc_fetch(self._h, orbit, 0, total.value, out.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(nw), None), "gc_fetch")
        return out

    def gc_fetch_starts(self, orbit: int, n: int) -> np.ndarray:
        out = np.zeros(n, dtype=START_DTYPE)
        nw = ctypes.c_uint64()
        self._check(self._L.gc_fetch_starts(self._h, orbit, 0, n, out.ctypes.data_as(ctypes.c_void_p),
                                            ctypes.byref(nw)), "gc_fetch_starts")
        return out[:nw.value]

    def gc_fetch_state(self, orbit: int, key_hi: int, key_lo: int) -> np.ndarray:
        ext = self.extent[orbit]
        out = np.empty(int(np.prod(ext)), dtype=np.float64)
        self._check(self._L.gc_fetch_state(self._h, orbit, int(key_hi), int(key_lo),
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "gc_fetch_state")
        return out

    def gc_fetch_start_state(self, orbit: int, start_id: int) -> np.ndarray:
        ext = self.extent[orbit]
        out = np.empty(int(np.prod(ext)), dtype=np.float64)
        self._check(self._L.gc_fetch_start_state(self._h, orbit, start_id,
                                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "gc_fetch_start_state")
        return out

    def gc_release(self, orbit: int):
        self._check(self._L.gc_release(self._h, orbit), "gc_release")
        self.extent.pop(orbit, None)

    def gc_kernel_time_ms(self, orbit: int) -> float:
        v = ctypes.c_double()
        self._check(self._L.gc_kernel_time_ms(self._h, orbit, ctypes.byref(v)), "gc_kernel_time_ms")
        return v.value

    def gc_launch_bytes(self, orbit: int, n_starts: int, params: SolveParams | None = None) -> int:
        p = (params or SolveParams()).c()
        b = ctypes.c_uint64()
        self._check(self._L.gc_launch_bytes(self._h, orbit, n_starts, ctypes.byref(p), ctypes.byref(b)),
                    "gc_launch_bytes")
        return b.value

    def gc_memory_info(self) -> dict:
        b, u, q = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self._L.gc_memory_info(self._h, ctypes.byref(b), ctypes.byref(u), ctypes.byref(q)),
                    "gc_memory_info")
        return {"budget": b.value, "in_use": u.value, "queued": q.value}

    def gc_autotune(self, orbit: int, n_starts: int, params: SolveParams | None = None) -> dict:
        p = (params or SolveParams()).c()
        r = gc_tune_result()
        self._check(self._L.gc_autotune(self._h, orbit, n_starts, ctypes.byref(p), ctypes.byref(r)), "gc_autotune")
        return {"relax_variant": r.relax_variant, "post_block": r.post_block,
                "post_sites_per_thread": r.post_sites_per_thread, "relax_ms": r.relax_ms, "post_ms": r.post_ms}

    def gc_saturation(self, orbit: int, sample_sizes, in_region_only: bool = False) -> np.ndarray:
        n = np.ascontiguousarray(sample_sizes, dtype=np.uint64)
        out = np.zeros(n.size, dtype=np.uint64)
        self._check(self._L.gc_saturation(self._h, orbit, int(n.size),
                                          n.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), int(in_region_only),
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), "gc_saturation")
        return out

    def gc_paper_saturation(self, orbit: int, sample_sizes) -> np.ndarray:
        n = np.ascontiguousarray(sample_sizes, dtype=np.uint64)
        out = np.zeros(n.size, dtype=np.uint64)
        self._check(self._L.gc_paper_saturation(self._h, orbit, int(n.size),
                                                n.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
                    "gc_paper_saturation")
        return out

    def gc_launch_static(self, orbit: int, n_starts: int, params: SolveParams | None, hip_stream: int,
                         copies_dev: int, copies_cap: int, n_copies_dev: int, counters_dev: int = 0):
        """Device pointers (integers) owned by the caller; enqueues and returns."""
        p = (params or SolveParams()).c()
        self._check(self._L.gc_launch_static(self._h, orbit, n_starts, ctypes.byref(p), hip_stream or None,
                                             copies_dev, copies_cap, n_copies_dev, counters_dev or None),
                    "gc_launch_static")

    def gc_last_error(self) -> str:
        buf = ctypes.create_string_buffer(512)
        self._L.gc_last_error(self._h, buf, 512)
        return buf.value.decode(errors="replace")

    # -- convenience: one full enumeration ----------------------------------
    def enumerate(self, orbit: int, n_starts: int, params: SolveParams | None = None, timeout_ms: int = -1):
        self.gc_launch(orbit, n_starts, params)
        if self.gc_wait(orbit, timeout_ms) != GC_OK:
            raise GcError(GC_ETIMEOUT, "gc_wait")
        return self.gc_fetch(orbit)
