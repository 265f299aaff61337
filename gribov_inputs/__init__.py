"""Seeded synthetic inputs for the Gribov-copy enumerator.

This module only draws random numbers and names workloads.  It holds none of
the method's arithmetic (no sweep, functional, key or eigenvalue code), so the
oracle under ``oracle/`` and the HIP path can both take their inputs from it
without sharing any computation.

Orbits are hot (random) gauge fields in the strong-coupling limit beta = 0:
every link angle is drawn independently and uniformly (Sec. I, paragraph on
compact U(1); Sec. III, last paragraph).  The counter map is fixed here so that
an orbit is a pure function of (seed, orbit_index, lattice shape):

* generator: Philox4x64-10 (Salmon et al., SC'11), as shipped by numpy;
* link l = mu*V + i draws block counter (l // 4, orbit_index, 0x4F, 0) under
  key (seed, 0) and uses output word l % 4;
* a 64-bit draw r becomes u = (r >> 11) * 2**-53 in [0, 1) and the angle
  fl(fl(u * 2pi) - pi) in [-pi, pi), with no fused multiply-add.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi
PI = math.pi
ORBIT_TAG = 0x4F
CONFIG4_TAG = 0x43
ARRIVAL_TAG = 0x41

_M64 = (1 << 64) - 1


def volume(extent) -> int:
    v = 1
    for n in extent:
        v *= int(n)
    return v


def _philox_blocks(key0: int, key1: int, ctr, n_blocks: int) -> np.ndarray:
    """Philox4x64-10 outputs for counters ctr, ctr+1, ... (word 0 increments).

    numpy's generator increments its 256-bit counter before producing each
    block, so it is seeded with ctr - 1 to make its first block use ctr.
    """
    c = sum((int(w) & _M64) << (64 * k) for k, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * k)) & _M64 for k in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([key0 & _M64, key1 & _M64], dtype=np.uint64), counter=words)
    return bg.random_raw(4 * n_blocks).astype(np.uint64)


def uniform_angle(raw: np.ndarray) -> np.ndarray:
    """Map 64-bit draws to angles in [-pi, pi): fl(fl(u*2pi) - pi)."""
    u = (raw >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    t = u * TWO_PI
    return t - PI


def orbit_angles(extent, seed: int = 0, orbit_index: int = 0) -> np.ndarray:
    """Hot orbit: link angles phi[mu][i], float64, shape (dim, V), uniform on [-pi, pi)."""
    extent = [int(n) for n in extent]
    dim = len(extent)
    V = volume(extent)
    n_links = dim * V
    n_blocks = (n_links + 3) // 4
    raw = _philox_blocks(seed, 0, (0, orbit_index, ORBIT_TAG, 0), n_blocks)[:n_links]
    return uniform_angle(raw).reshape(dim, V)


SU2_TAG = 0x55


def su2_links(extent, seed: int = 0, orbit_index: int = 0) -> np.ndarray:
    """Hot SU(2) configuration (beta = 0): every link Haar-random, as a unit
    quaternion (a0, a1, a2, a3) for U = a0 + i (a1 s1 + a2 s2 + a3 s3);
    float64, shape (dim, V, 4).  Link l = mu*V + i takes four normal
    deviates (Box-Muller on the uniforms of counter (0, orbit_index, 0x55, 0)
    onwards under key (seed, 2), eight uniforms per link) scaled to unit
    length, which is the uniform distribution on the 3-sphere."""
    extent = [int(n) for n in extent]
    dim, V = len(extent), volume(extent)
    n = dim * V
    u = uniform01(seed, (0, orbit_index, SU2_TAG, 0), 8 * n).reshape(n, 4, 2)
    r = np.sqrt(-2.0 * np.log1p(-u[..., 0]))
    z = np.where(np.arange(4) % 2 == 0, r * np.cos(TWO_PI * u[..., 1]), r * np.sin(TWO_PI * u[..., 1]))
    z /= np.sqrt((z * z).sum(axis=1, keepdims=True))
    return z.reshape(dim, V, 4)


def cold_orbit(extent) -> np.ndarray:
    """Trivial orbit: every link angle zero (Sec. I)."""
    return np.zeros((len(extent), volume(extent)), dtype=np.float64)


def constant_orbit(extent, c) -> np.ndarray:
    """Orbit with phi[mu][i] = c[mu] for every site."""
    V = volume(extent)
    return np.repeat(np.asarray(c, dtype=np.float64)[:, None], V, axis=1)


def uniform01(seed: int, ctr, n: int) -> np.ndarray:
    raw = _philox_blocks(seed, 2, ctr, (n + 3) // 4)[:n]
    return (raw >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ---------------------------------------------------------------------------
# Named workloads.  Each is stated with its sizes; start angles are drawn by
# each side's own Philox from (start_seed, start_id, orbit_index).
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    extent: tuple
    n_starts: int
    omega: float
    precision: str          # "fp64" or "mixed"
    eps64: float = 1e-14
    eps32: float = 1e-6
    seed: int = 0
    orbit_index: int = 0
    start_seed: int = 0
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    # 2D 4x4, 1000 starts, overrelaxation 1.7, FP64, with the FP-operator filter.
    "u1_2d_4x4_or": Workload("u1_2d_4x4_or", (4, 4), 1000, 1.7, "fp64"),
    # 4D 4^4, 1e5 starts, plain relaxation (omega = 1), FP64.
    "u1_4d_4x4x4x4_relax": Workload("u1_4d_4x4x4x4_relax", (4, 4, 4, 4), 100_000, 1.0, "fp64"),
    # 4D 6^4 and 3D 10^3, 1e6 starts, FP32 overrelaxation to 1e-6 then FP64 polish,
    # and the same orbits and starts in double precision throughout.
    "u1_4d_6x6x6x6_mixed": Workload("u1_4d_6x6x6x6_mixed", (6, 6, 6, 6), 1_000_000, 1.7, "mixed"),
    "u1_3d_10x10x10_mixed": Workload("u1_3d_10x10x10_mixed", (10, 10, 10), 1_000_000, 1.7, "mixed"),
    "u1_4d_6x6x6x6_fp64": Workload("u1_4d_6x6x6x6_fp64", (6, 6, 6, 6), 1_000_000, 1.7, "fp64"),
    "u1_3d_10x10x10_fp64": Workload("u1_3d_10x10x10_fp64", (10, 10, 10), 1_000_000, 1.7, "fp64"),
}

# Shapes of the uneven multi-orbit batch (even extents only).
BATCH_SHAPES = [(8, 8), (10, 10), (12, 12), (14, 14), (16, 16),
                (6, 6, 6), (8, 8, 8), (4, 4, 4, 4), (6, 6, 6, 6)]


def uneven_batch(n_orbits: int = 32, seed: int = 0, lo: float = 1e3, hi: float = 1e5):
    """Uneven multi-orbit batch: orbit k has shape BATCH_SHAPES[k % 9] and
    round(lo * (hi/lo)**u_k) starts, u_k uniform from Philox key (seed, 2),
    counter (k, 0, 0, 0x43)."""
    out = []
    span = math.log10(hi / lo)
    for k in range(n_orbits):
        u = float(uniform01(seed, (k, 0, 0, CONFIG4_TAG), 1)[0])
        n = int(round(lo * 10.0 ** (span * u)))
        out.append(dict(extent=BATCH_SHAPES[k % len(BATCH_SHAPES)], n_starts=n,
                        seed=seed, orbit_index=k))
    return out


def poisson_requests(n_requests: int, rate_per_s: float, seed: int = 0,
                     extra_shapes=(((8, 8, 8, 8), 10_000),)):
    """Serving stream: exponential inter-arrival times at rate_per_s; request j
    takes a shape uniformly from BATCH_SHAPES plus extra_shapes, with a
    log-uniform start count in [1e3, 1e5] for batch shapes."""
    u = uniform01(seed, (0, 0, 0, ARRIVAL_TAG), 3 * n_requests).reshape(n_requests, 3)
    shapes = list(BATCH_SHAPES) + [s for s, _ in extra_shapes]
    t = 0.0
    reqs = []
    for j in range(n_requests):
        t += -math.log(1.0 - u[j, 0]) / rate_per_s
        si = min(int(u[j, 1] * len(shapes)), len(shapes) - 1)
        if si < len(BATCH_SHAPES):
            n = int(round(1e3 * 10.0 ** (2.0 * u[j, 2])))
        else:
            n = extra_shapes[si - len(BATCH_SHAPES)][1]
        reqs.append(dict(t_arrive=t, extent=shapes[si], n_starts=n, seed=seed,
                         orbit_index=1000 + j))
    return reqs
