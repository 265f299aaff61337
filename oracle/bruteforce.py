"""Brute-force stationary points of eq. (3) on tiny lattices -- TEST INFRASTRUCTURE.

Finds (ideally all) stationary points of F_phi(theta), eq. (3), with the
global phase removed by holding the last site's angle at zero (Sec. I,
compact U(1) paragraph), by Newton's method from a grid or a random cloud
of starting points on the torus T^(V-1).  Each point is classified by the
Morse index of the reduced Hessian (the FP operator with the fixed site's row
and column removed).  For a complete set, eq. (2) requires
sum over stationary points of sign det M_FP = chi(S^1)^(V-1) = 0,
and the minima (index 0) are the copies of the first Gribov region.

Plain numpy; independent of the C oracle (own gradient and Hessian from the
link angles).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def _geometry(extent):
    extent = [int(n) for n in extent]
    d = len(extent)
    V = int(np.prod(extent))
    strides = [1]
    for n in extent[:-1]:
        strides.append(strides[-1] * n)
    coords = np.array([[(i // strides[mu]) % extent[mu] for mu in range(d)] for i in range(V)])
    fwd = np.zeros((d, V), dtype=np.int64)
    for mu in range(d):
        for i in range(V):
            x = coords[i].copy()
            x[mu] = (x[mu] + 1) % extent[mu]
            fwd[mu, i] = int(np.dot(x, strides))
    return d, V, fwd


class Landscape:
    """F, gradient and Hessian of eq. (3) for one orbit, as functions of theta."""

    def __init__(self, extent, phi):
        self.d, self.V, self.fwd = _geometry(extent)
        self.phi = np.asarray(phi, dtype=np.float64).reshape(self.d, self.V)
        base = np.repeat(np.arange(self.V)[None, :], self.d, axis=0)
        self.base = base.reshape(-1)
        self.head = self.fwd.reshape(-1)
        self.phil = self.phi.reshape(-1)

    def link_angles(self, theta):
        return self.phil + theta[self.head] - theta[self.base]

    def F(self, theta):
        return float(np.sum(1.0 - np.cos(self.link_angles(theta))))

    def grad(self, theta):
        s = np.sin(self.link_angles(theta))
        g = np.zeros(self.V)
        np.add.at(g, self.head, s)      # dF/dtheta_head of (1 - cos a) = +sin a
        np.add.at(g, self.base, -s)     # dF/dtheta_base = -sin a
        return g

    def hessian(self, theta):
        c = np.cos(self.link_angles(theta))
        H = np.zeros((self.V, self.V))
        np.add.at(H, (self.base, self.base), c)
        np.add.at(H, (self.head, self.head), c)
        np.add.at(H, (self.base, self.head), -c)
        np.add.at(H, (self.head, self.base), -c)
        return H


def newton(land: Landscape, theta0, max_iter: int = 60, tol: float = 1e-12):
    """Newton on the reduced variables theta_0..theta_{V-2}; theta_{V-1} = 0."""
    th = np.array(theta0, dtype=np.float64)
    th[-1] = 0.0
    for _ in range(max_iter):
        g = land.grad(th)[:-1]
        if np.max(np.abs(g)) < tol:
            return th
        H = land.hessian(th)[:-1, :-1]
        try:
            step = np.linalg.solve(H, g)
        except np.linalg.LinAlgError:
            return None
        if not np.all(np.isfinite(step)):
            return None
        th[:-1] -= step
    g = land.grad(th)[:-1]
    return th if np.max(np.abs(g)) < tol else None


def canonical(theta):
    """Angles wrapped to (-pi, pi] (theta_{V-1} is 0 already)."""
    return np.angle(np.exp(1j * theta))


def stationary_points(extent, phi, starts):
    """Distinct stationary points reached by Newton from the given starts.

    Returns list of dicts {theta, F, index}; points are distinct if their
    canonical angles differ by more than 1e-7 anywhere (mod 2 pi)."""
    land = Landscape(extent, phi)
    pts = []
    seen = {}
    for t0 in starts:
        th = newton(land, t0)
        if th is None:
            continue
        c = canonical(th)
        # Bucket by coarse rounding of (cos, sin) (no wrap ambiguity), then
        # confirm with a fine comparison inside the bucket.
        b = tuple(np.rint(np.concatenate([np.cos(c), np.sin(c)]) * 1e4).astype(np.int64))
        dup = False
        for p in seen.get(b, []):
            diff = np.angle(np.exp(1j * (c - p["theta"])))
            if np.max(np.abs(diff)) < 1e-7:
                dup = True
                break
        # Newton lands within ~1e-12 of a point, so two landings on one point
        # straddle a 1e-4 rounding edge with probability ~1e-8.
        if dup:
            continue
        H = land.hessian(c)[:-1, :-1]
        ev = np.linalg.eigvalsh(H)
        pt = dict(theta=c, F=land.F(c), index=int(np.sum(ev < 0)),
                  min_abs_eig=float(np.min(np.abs(ev))))
        pts.append(pt)
        seen.setdefault(b, []).append(pt)
    return pts


def grid_starts(V: int, n_per_axis: int):
    ax = -math.pi + (np.arange(n_per_axis) + 0.5) * TWO_PI / n_per_axis
    for p in itertools.product(ax, repeat=V - 1):
        yield np.array(list(p) + [0.0])


def random_starts(V: int, n: int, seed: int = 1234):
    rng = np.random.Generator(np.random.Philox(seed))
    for _ in range(n):
        t = rng.uniform(-math.pi, math.pi, V)
        t[-1] = 0.0
        yield t


def euler_sum(points) -> int:
    """sum over stationary points of sign det(reduced M_FP) = sum (-1)^index (eq. (2))."""
    return int(sum((-1) ** p["index"] for p in points))
