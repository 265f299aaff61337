"""Oracle for the Gribov-copy enumerator -- TEST INFRASTRUCTURE ONLY.

Plain double-precision CPU reference.  Only ``tests/``, the smoke check and
the benchmark's CPU-baseline leg may import this module; the product path
never does, and the two share no code.

The per-start relaxation, the functional and the integer key run in
``gribov_oracle.c`` (plain C, compiled without floating-point contraction).
This module adds, in numpy:

* the Faddeev-Popov operator M_FP, the Hessian of eq. (3) in theta
  (Sec. I, lattice Landau gauge paragraph), assembled densely as
  B^T diag(cos a) B from the link-site incidence matrix B, and its spectrum by
  LAPACK (numpy.linalg.eigvalsh);
* the first-Gribov-region test (abstract; Sec. I: minima, i.e. M_FP positive
  semidefinite with only the constant zero mode);
* the copy table: distinct minima keyed by the integer key, with hit counts,
  the lowest start id reaching each, its representative start (lowest id at the
  lowest functional value of the class), and the paper's own count of distinct
  values of x at resolution 1e-8 (Sec. III, last paragraphs).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gribov_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CONVERGED, NONCONVERGED, BADNUM = 1, 2, 3
FLAG_IN_REGION, FLAG_SINGULAR, FLAG_SADDLE, FLAG_COLLISION = 1, 2, 4, 8
LAMBDA_TOL = 1e-6

RECORD_DTYPE = np.dtype([
    ("status", np.int32), ("sweeps32", np.int32), ("sweeps64", np.int32), ("n_elems", np.int32),
    ("F", np.float64), ("x", np.float64), ("D", np.float64), ("cut_margin", np.float64),
    ("key_hi", np.uint64), ("key_lo", np.uint64), ("paper_X", np.uint32), ("key_overflow", np.int32),
])


class _Params(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("eps32", ctypes.c_double), ("eps64", ctypes.c_double),
                ("precision", ctypes.c_int32), ("stop_norm", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("fixed", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int64), ("start_seed", ctypes.c_uint64),
                ("orbit_index", ctypes.c_uint64)]


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, -O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        L.oracle_philox4x64_10.argtypes = [P(ctypes.c_uint64), P(ctypes.c_uint64), P(ctypes.c_uint64)]
        L.oracle_mix64.argtypes = [ctypes.c_uint64]
        L.oracle_mix64.restype = ctypes.c_uint64
        L.oracle_start_angles.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_int64, P(ctypes.c_double)]
        L.oracle_key_length.argtypes = [ctypes.c_int, P(ctypes.c_int)]
        L.oracle_key_length.restype = ctypes.c_int64
        L.oracle_solve.argtypes = [ctypes.c_int, P(ctypes.c_int), P(ctypes.c_double), P(ctypes.c_uint64),
                                   ctypes.c_int64, P(_Params), P(ctypes.c_double), ctypes.c_int,
                                   ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_int32)]
        L.oracle_observe.argtypes = [ctypes.c_int, P(ctypes.c_int), P(ctypes.c_double), P(ctypes.c_double),
                                     ctypes.c_void_p, P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_double)]
        L.oracle_colouring.argtypes = [ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int32)]
        L.oracle_neighbours.argtypes = [ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int32), P(ctypes.c_int32)]
        assert L.oracle_record_size() == RECORD_DTYPE.itemsize
        assert L.oracle_params_size() == ctypes.sizeof(_Params)
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ext(extent):
    e = np.zeros(4, dtype=np.int32)
    e[:len(extent)] = extent
    return e, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def volume(extent) -> int:
    return int(np.prod(extent))


# --------------------------------------------------------------------------
# Small primitives (exposed for pinning against published values)
# --------------------------------------------------------------------------

def philox(ctr, key):
    c = (ctypes.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(x) for x in key])
    o = (ctypes.c_uint64 * 4)()
    lib().oracle_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def mix64(z: int) -> int:
    return int(lib().oracle_mix64(ctypes.c_uint64(z & ((1 << 64) - 1))))


def start_angles(start_seed: int, start_id: int, orbit_index: int, V: int) -> np.ndarray:
    out = np.empty(V, dtype=np.float64)
    lib().oracle_start_angles(start_seed, start_id, orbit_index, V, _dp(out))
    return out


def colouring(extent):
    e, ep = _ext(extent)
    col = np.empty(volume(extent), dtype=np.int32)
    K = lib().oracle_colouring(len(extent), ep, col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return K, col


def neighbours(extent):
    e, ep = _ext(extent)
    d, V = len(extent), volume(extent)
    fwd = np.empty((d, V), dtype=np.int32)
    bwd = np.empty((d, V), dtype=np.int32)
    P = ctypes.POINTER(ctypes.c_int32)
    rc = lib().oracle_neighbours(d, ep, fwd.ctypes.data_as(P), bwd.ctypes.data_as(P))
    assert rc == 0
    return fwd, bwd


def key_length(extent) -> int:
    e, ep = _ext(extent)
    return int(lib().oracle_key_length(len(extent), ep))


# --------------------------------------------------------------------------
# Relaxation (C) -- eqs. (4)-(5) in the convention of eq. (3)
# --------------------------------------------------------------------------

@dataclass
class SolveParams:
    omega: float = 1.0
    precision: str = "fp64"        # "fp64" or "mixed"
    eps32: float = 1e-6
    eps64: float = 1e-14
    stop_norm: str = "mean_sq"     # or "max_abs" (the paper's rule)
    check_every: int = 1
    max_sweeps: int = 100_000
    start_seed: int = 0
    orbit_index: int = 0
    fixed: bool = False            # run exactly max_sweeps double sweeps (batch-synchronous second pass)

    def c(self) -> _Params:
        return _Params(self.omega, self.eps32, self.eps64, 1 if self.precision == "mixed" else 0,
                       1 if self.stop_norm == "max_abs" else 0, self.check_every, 1 if self.fixed else 0,
                       self.max_sweeps, self.start_seed, self.orbit_index)


def twisted(extent, phi, antiperiodic: int = 0) -> np.ndarray:
    """Link angles of the periodic problem equivalent to antiperiodic gauge
    transformations in the directions of the bit mask (Sec. II names
    antiperiodic boundary conditions).  With g_{x + N_mu e_mu} = -g_x the
    term of a link (x, mu) with x_mu = N_mu - 1 reads
    Re(conj(g_x) U (-g_{x'})) = Re(conj(g_x) (-U) g_{x'}), x' the periodic
    image: the link angle gains pi."""
    d, V = len(extent), volume(extent)
    out = np.array(phi, dtype=np.float64).reshape(d, V).copy()
    if not antiperiodic:
        return out
    idx = np.arange(V)
    stride = 1
    for mu, n in enumerate(extent):
        x = (idx // stride) % n
        if (antiperiodic >> mu) & 1:
            out[mu, x == n - 1] += math.pi
        stride *= n
    return out


def solve(extent, phi, start_ids, params: SolveParams, theta_init=None, threads: int = 0,
          want_state: bool = False, want_payload: bool = False):
    """Relax the listed starts.  Returns (records, g or None, payload or None).

    g has shape (n, V, 2) (final Re, Im of g_i); payload (n, m) int32."""
    e, ep = _ext(extent)
    d, V = len(extent), volume(extent)
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(d, V)
    ids = np.ascontiguousarray(start_ids, dtype=np.uint64)
    n = ids.size
    rec = np.zeros(n, dtype=RECORD_DTYPE)
    g = np.empty((n, V, 2), dtype=np.float64) if want_state else None
    m = key_length(extent)
    pay = np.empty((n, m), dtype=np.int32) if want_payload else None
    th = None
    if theta_init is not None:
        th = np.ascontiguousarray(theta_init, dtype=np.float64).reshape(n, V)
    prm = params.c()
    rc = lib().oracle_solve(d, ep, _dp(phi), ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n,
                            ctypes.byref(prm), _dp(th), threads, rec.ctypes.data_as(ctypes.c_void_p),
                            _dp(g), pay.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if pay is not None else None)
    if rc != 0:
        raise ValueError("oracle_solve: unsupported lattice %r (rc=%d)" % (tuple(extent), rc))
    return rec, g, pay


def observe(extent, phi, theta):
    """Functional, key and link data of the state g = exp(i theta) (no relaxation)."""
    e, ep = _ext(extent)
    d, V = len(extent), volume(extent)
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(d, V)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    rec = np.zeros(1, dtype=RECORD_DTYPE)
    m = key_length(extent)
    pay = np.empty(m, dtype=np.int32)
    a = np.empty((d, V), dtype=np.float64)
    w = np.empty((d, V), dtype=np.float64)
    rc = lib().oracle_observe(d, ep, _dp(phi), _dp(theta), rec.ctypes.data_as(ctypes.c_void_p),
                              pay.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(a), _dp(w))
    assert rc == 0
    return rec[0], pay, a, w


def theta_of(g) -> np.ndarray:
    """theta_i = arg g_i for a state of shape (V, 2)."""
    return np.arctan2(g[:, 1], g[:, 0])


# --------------------------------------------------------------------------
# Faddeev-Popov operator (Hessian of eq. (3)) and the first Gribov region
# --------------------------------------------------------------------------

def incidence(extent) -> np.ndarray:
    """B[l, site]: a_l = phi_l + theta_{i+mu} - theta_i, so dA_l/dtheta = +1 at
    the forward end and -1 at the base (rows l = mu*V + i)."""
    d, V = len(extent), volume(extent)
    fwd, _ = neighbours(extent)
    B = np.zeros((d * V, V), dtype=np.float64)
    for mu in range(d):
        for i in range(V):
            l = mu * V + i
            B[l, i] -= 1.0
            B[l, fwd[mu, i]] += 1.0
    return B


def fp_operator(extent, w) -> np.ndarray:
    """M_FP = B^T diag(w) B with w_l = cos a_l (the Hessian of eq. (3))."""
    B = incidence(extent)
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    return B.T @ (w[:, None] * B)


def fp_spectrum(extent, w):
    """(lambda_zero, lambda2, lambda_max).

    M always annihilates the constant vector.  lambda2 is the lowest
    eigenvalue of M on the complement of the constant vector, computed
    densely as the lowest eigenvalue of M + sigma 11^T/V with sigma above
    every eigenvalue of M (|lambda| <= 4d by Gershgorin).  lambda_zero is the
    eigenvalue of M nearest to zero, for the zero-mode check."""
    d, V = len(extent), volume(extent)
    M = fp_operator(extent, w)
    ev = np.linalg.eigvalsh(M)
    sigma = 4.0 * d + 1.0
    ev_shift = np.linalg.eigvalsh(M + sigma / V * np.ones((V, V)))
    lam0 = ev[np.argmin(np.abs(ev))]
    return float(lam0), float(ev_shift[0]), float(ev[-1])


def region_flags(lam2: float, tol: float = LAMBDA_TOL) -> int:
    if lam2 > tol:
        return FLAG_IN_REGION
    if lam2 < -tol:
        return FLAG_SADDLE
    return FLAG_SINGULAR


# --------------------------------------------------------------------------
# Enumeration of one orbit: per-start solves + copy table
# --------------------------------------------------------------------------

F_SPREAD_PER_SITE = 1e-9


def solve_sync(extent, phi, start_ids, params: SolveParams, batch: int, threads: int = 0,
               want_state: bool = False):
    """The paper's batch-synchronous stop (Sec. III: one stopping test over
    all samples relaxed together): the starts are taken in batches of
    `batch` consecutive entries of start_ids; every start of a batch runs
    the largest number of sweeps any start of the batch needs to stop on its
    own, and is converged if its norm is below eps64 after them.  FP64."""
    assert params.precision == "fp64"
    ids = np.ascontiguousarray(start_ids, dtype=np.uint64)
    first, _, _ = solve(extent, phi, ids, params, threads=threads)
    rec = np.zeros(ids.size, dtype=RECORD_DTYPE)
    V = volume(extent)
    g = np.empty((ids.size, V, 2)) if want_state else None
    for lo in range(0, ids.size, batch):
        hi = min(ids.size, lo + batch)
        T = int(first["sweeps64"][lo:hi].max())
        p2 = SolveParams(**{**params.__dict__, "max_sweeps": T, "fixed": True})
        r, gg, _ = solve(extent, phi, ids[lo:hi], p2, threads=threads, want_state=want_state)
        rec[lo:hi] = r
        if want_state:
            g[lo:hi] = gg
    return rec, g


def enumerate_copies(extent, phi, start_ids, params: SolveParams, threads: int = 0,
                     with_lambda: bool = True, lambda_keys=None, sync_batch: int = 0):
    """Run the listed starts and build the copy table.

    A key can be reached by starts that stopped at different stationary
    points of the same wrap class: relaxation may halt next to a saddle when
    the divergence is already below the threshold there.  Copies are minima
    (first Gribov region), so a copy is represented by the lowest start id
    among its hits whose F lies within 1e-9 per site of the lowest F reaching
    the key; F and lambda2 are that start's.  first_start is the lowest id
    over all hits; a spread of F above 1e-9 per site sets FLAG_COLLISION.

    lambda_keys: None (all copies) or a set of keys whose lambda2 is wanted.
    Returns dict with 'records' (per start), 'table' {(key_hi, key_lo): entry},
    'paper_count' (distinct trunc(x*1e8) over converged starts)."""
    ids = np.ascontiguousarray(start_ids, dtype=np.uint64)
    if sync_batch:
        rec, g = solve_sync(extent, phi, ids, params, sync_batch, threads=threads, want_state=with_lambda)
    else:
        rec, g, _ = solve(extent, phi, ids, params, threads=threads, want_state=with_lambda)
    V = volume(extent)
    hits = {}
    for s in range(ids.size):
        r = rec[s]
        if r["status"] != CONVERGED:
            continue
        hits.setdefault((int(r["key_hi"]), int(r["key_lo"])), []).append(s)
    table = {}
    for k, idx in hits.items():
        Fs = np.array([rec["F"][s] for s in idx])
        sids = np.array([int(ids[s]) for s in idx], dtype=np.uint64)
        F_min, F_max = float(Fs.min()), float(Fs.max())
        near = Fs - F_min <= F_SPREAD_PER_SITE * V
        rep = idx[int(np.argmin(np.where(near, sids, np.iinfo(np.uint64).max)))]
        e = dict(hits=len(idx), first_start=int(sids.min()), rep_start=int(ids[rep]), rep_index=rep,
                 F=float(rec["F"][rep]), F_min=F_min, F_max=F_max)
        flags = 0
        if with_lambda and (lambda_keys is None or k in lambda_keys):
            _, _, _, w = observe(extent, phi, theta_of(g[rep]))
            lam0, lam2, lmax = fp_spectrum(extent, w)
            e["lambda2"], e["lambda_zero"], e["lambda_max"] = lam2, lam0, lmax
            flags |= region_flags(lam2)
        if (F_max - F_min) / V > F_SPREAD_PER_SITE:
            flags |= FLAG_COLLISION
        e["flags"] = flags
        e["x"] = e["F"] / (len(extent) * V)
        table[k] = e
    conv = rec["status"] == CONVERGED
    paper_count = int(np.unique(rec["paper_X"][conv]).size)
    return dict(records=rec, table=table, paper_count=paper_count, state=g)


# --------------------------------------------------------------------------
# Distributions of the minima over orbits (Sec. IV.B)
# --------------------------------------------------------------------------

HIST_X, HIST_REL = 0, 1
HIST_COPIES, HIST_STARTS = 0, 1


def histogram(copies, dim: int, V: int, quantity: int, weight: int, require_flags: int,
              lo: float, hi: float, n_bins: int) -> np.ndarray:
    """Counts of one orbit's minima in n_bins equal bins of [lo, hi), with an
    underflow count first and an overflow count last (n_bins + 2 entries).

    copies: iterable of dicts with 'F', 'flags', 'hits' (a copy table's entries).
    Only copies carrying every flag of require_flags count.  The binned value
    is x = F / (d V) (quantity HIST_X; the functional per link, eq. (3)) or the
    deviation from the orbit's global minimum (F - F_g) / F_g with F_g the
    lowest F among the counted copies (quantity HIST_REL).  A copy adds 1
    (HIST_COPIES) or its number of hits (HIST_STARTS).  A value v falls in bin
    1 + floor(((v - lo) / (hi - lo)) * n_bins), evaluated in double precision
    in that order and capped at the last bin; v < lo (or NaN) underflows and
    v >= hi overflows."""
    counted = [e for e in copies if (int(e["flags"]) & require_flags) == require_flags]
    out = np.zeros(n_bins + 2, dtype=np.uint64)
    if not counted:
        return out
    F_g = min(float(e["F"]) for e in counted)
    for e in counted:
        F = float(e["F"])
        v = F / float(dim * V) if quantity == HIST_X else (F - F_g) / F_g
        if not v >= lo:
            b = 0
        elif not v < hi:
            b = n_bins + 1
        else:
            b = 1 + min(n_bins - 1, int(math.floor(((v - lo) / (hi - lo)) * n_bins)))
        out[b] += int(e["hits"]) if weight == HIST_STARTS else 1
    return out


# --------------------------------------------------------------------------
# SU(2) configurations through the maximal Abelian reduction.  Sec. I states
# the Landau functional for SU(N_c) (eq. (1)) and argues that the Neuberger
# problem of SU(N_c) lies in the maximal Abelian subgroup U(1)^{N_c-1}, the
# coset part being free of it; the U(1) copies are the ones enumerated.  An
# SU(2) configuration is therefore gauge-fixed on the coset SU(2)/U(1) to the
# maximal Abelian gauge (the reading: maximise R = sum_{x,mu} 1/2 Tr(s3 U' s3
# U'^dagger), U' = g_x U_{x,mu} g_{x+mu}^dagger, by local maximisation colour
# by colour), and the diagonal phases of U' form the compact U(1) orbit.
# Quaternions q = (q0, q1, q2, q3) stand for q0 + i (q1 s1 + q2 s2 + q3 s3).
# --------------------------------------------------------------------------

def q_mul(p, q):
    """Product of quaternions (..., 4): (i s_a)(i s_b) = -delta_ab - i eps_abc s_c."""
    p0, p1, p2, p3 = p[..., 0], p[..., 1], p[..., 2], p[..., 3]
    r0, r1, r2, r3 = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([p0 * r0 - p1 * r1 - p2 * r2 - p3 * r3,
                     p0 * r1 + r0 * p1 - (p2 * r3 - p3 * r2),
                     p0 * r2 + r0 * p2 - (p3 * r1 - p1 * r3),
                     p0 * r3 + r0 * p3 - (p1 * r2 - p2 * r1)], axis=-1)


def q_conj(q):
    """Inverse of a unit quaternion (the Hermitian conjugate)."""
    return q * np.array([1.0, -1.0, -1.0, -1.0])


def q_rot3(q):
    """b with Q s3 Q^dagger = b . s for Q = q: b3 = |alpha|^2 - |beta|^2 and
    b1 - i b2 = -2 alpha beta for Q = [[alpha, beta], [-conj(beta), conj(alpha)]],
    alpha = q0 + i q3, beta = q2 + i q1."""
    q0, q1, q2, q3 = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([-2.0 * (q0 * q2 - q1 * q3), 2.0 * (q0 * q1 + q2 * q3),
                     q0 * q0 + q3 * q3 - q1 * q1 - q2 * q2], axis=-1)


def q_from_axis3(n):
    """The gauge transformation g with g^dagger s3 g = n . s whose diagonal
    element is real and non-negative (h = g^dagger: alpha = sqrt((1 + n3)/2),
    beta = -(n1 - i n2)/(2 alpha); alpha = 0, beta = 1 at n3 = -1)."""
    a = np.sqrt(0.5 * (1.0 + n[..., 2]))
    safe = a > 0.0
    den = np.where(safe, 2.0 * a, 1.0)
    br = np.where(safe, -n[..., 0] / den, 1.0)
    bi = np.where(safe, n[..., 1] / den, 0.0)
    h = np.stack([a, bi, br, np.zeros_like(a)], axis=-1)   # alpha = h0 + i h3, beta = h2 + i h1
    return q_conj(h)


def mag_transformed(extent, links, g):
    """U'_{x,mu} = g_x U_{x,mu} g_{x+mu}^dagger, shape (dim, V, 4)."""
    fwd, _ = neighbours(extent)
    d = len(extent)
    return np.stack([q_mul(q_mul(g, links[mu]), q_conj(g[fwd[mu]])) for mu in range(d)])


def mag_project(extent, links, eps: float = 1e-20, max_sweeps: int = 100000, want_g: bool = False):
    """Maximal Abelian gauge by local maximisation and the Abelian projection.

    Sweeps update the sites of colour 0, then of colour 1 (even extents): at
    site x, R depends on g_x only through n . M, n . s = g_x^dagger s3 g_x and
    M = sum_mu [w_mu + y_mu] (mu ascending, forward then backward), with
    W = U_{x,mu} g_{x+mu}^dagger, w . s = W s3 W^dagger, and
    Y = g_{x-mu} U_{x-mu,mu}, y . s = Y^dagger s3 Y; so n = M/|M| (M = 0
    leaves g_x unchanged) and g_x = q_from_axis3(n).  D = (1/V) sum_x
    |n_x - n_x^old|^2 over a sweep; the reduction stops after the first sweep
    with D < eps.  Returns (phi [dim][V] = arg of the diagonal element q0 +
    i q3 of U', sweeps, R/(dim V), converged[, g])."""
    ext = [int(n) for n in extent]
    d, V = len(ext), volume(ext)
    if any(n % 2 for n in ext):
        raise ValueError("the maximal Abelian reduction needs even extents")
    links = np.asarray(links, dtype=np.float64).reshape(d, V, 4)
    fwd, bwd = neighbours(ext)
    coords = np.array(np.unravel_index(np.arange(V), ext[::-1]))[::-1]
    colour = coords.sum(axis=0) % 2
    sites = [np.nonzero(colour == c)[0] for c in (0, 1)]
    g = np.zeros((V, 4))
    g[:, 0] = 1.0
    sweeps, converged = 0, False
    while sweeps < max_sweeps:
        acc = 0.0
        for c in (0, 1):
            x = sites[c]
            M = np.zeros((x.size, 3))
            for mu in range(d):
                W = q_mul(links[mu, x], q_conj(g[fwd[mu, x]]))
                M = M + q_rot3(W)
                b = bwd[mu, x]
                Y = q_mul(g[b], links[mu, b])
                M = M + q_rot3(q_conj(Y))
            m2 = (M * M).sum(axis=1)
            ok = m2 > 0.0
            n = M / np.sqrt(np.where(ok, m2, 1.0))[:, None]
            old = q_rot3(q_conj(g[x]))
            new_g = np.where(ok[:, None], q_from_axis3(n), g[x])
            new_n = np.where(ok[:, None], n, old)
            acc += float(((new_n - old) ** 2).sum())
            g[x] = new_g
        sweeps += 1
        if acc / V < eps:
            converged = True
            break
    Up = mag_transformed(ext, links, g)
    R = float(q_rot3(Up)[..., 2].sum()) / (d * V)
    phi = np.arctan2(Up[..., 3], Up[..., 0])
    if want_g:
        return phi, sweeps, R, converged, g
    return phi, sweeps, R, converged
