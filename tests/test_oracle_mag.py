"""Pins of the oracle's maximal Abelian reduction of SU(2) configurations
(Sec. I: eq. (1) for SU(N_c); the Neuberger problem of SU(N_c) lies in the
maximal Abelian subgroup, whose U(1) copies are enumerated).

* Quaternion algebra against explicit 2x2 complex matrices (an independent
  route): products, Q s3 Q^dagger, the canonical transformation of an axis.
* An Abelian configuration (every link diagonal) is a fixed point: one sweep,
  R = 1, and the projection returns the link angles.
* The same configuration after a smooth SU(2) gauge transformation: the
  reduction recovers R = 1 and an Abelian field with the original plaquette
  angles (gauge invariants) modulo 2 pi.
* R never decreases from sweep to sweep, and the result is a local maximum.
"""
import math

import numpy as np
import pytest

import gribov_inputs as GI
from oracle import oracle as O

S1 = np.array([[0, 1], [1, 0]], dtype=complex)
S2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
S3 = np.array([[1, 0], [0, -1]], dtype=complex)


def mat(q):
    return q[0] * np.eye(2) + 1j * (q[1] * S1 + q[2] * S2 + q[3] * S3)


def rand_q(rng, n):
    z = rng.normal(size=(n, 4))
    return z / np.linalg.norm(z, axis=1, keepdims=True)


def test_quaternion_algebra_matches_matrices():
    rng = np.random.default_rng(1)
    p, q = rand_q(rng, 50), rand_q(rng, 50)
    r = O.q_mul(p, q)
    b = O.q_rot3(q)
    for k in range(50):
        assert np.allclose(mat(r[k]), mat(p[k]) @ mat(q[k]), atol=1e-14)
        Q = mat(q[k])
        assert np.allclose(Q @ S3 @ Q.conj().T, b[k, 0] * S1 + b[k, 1] * S2 + b[k, 2] * S3, atol=1e-14)
        assert np.allclose(mat(O.q_conj(q[k])), Q.conj().T, atol=1e-15)
    n = rand_q(rng, 50)[:, 1:]
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n = np.vstack([n, [0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    g = O.q_from_axis3(n)
    for k in range(len(n)):
        G = mat(g[k])
        assert np.allclose(G.conj().T @ S3 @ G, n[k, 0] * S1 + n[k, 1] * S2 + n[k, 2] * S3, atol=1e-14)
        h = G.conj().T
        assert abs(h[0, 0].imag) < 1e-15 and h[0, 0].real >= 0.0


def abelian_links(phi):
    return np.stack([np.cos(phi), np.zeros_like(phi), np.zeros_like(phi), np.sin(phi)], axis=-1)


@pytest.mark.parametrize("extent", [(4, 4), (6, 4), (4, 4, 4), (2, 2, 2, 2)])
def test_abelian_configuration_is_a_fixed_point(extent):
    phi = GI.orbit_angles(extent, 3, 1)
    out, sweeps, R, conv = O.mag_project(extent, abelian_links(phi))
    assert conv and sweeps == 1
    assert abs(R - 1.0) < 1e-15
    assert np.max(np.abs(np.angle(np.exp(1j * (out - phi))))) < 1e-15


def plaquette_angles(extent, phi):
    fwd, _ = O.neighbours(extent)
    d = len(extent)
    out = []
    for mu in range(d):
        for nu in range(mu + 1, d):
            out.append(phi[mu] + phi[nu][fwd[mu]] - phi[mu][fwd[nu]] - phi[nu])
    return np.array(out)


@pytest.mark.parametrize("extent", [(4, 4), (4, 4, 4), (4, 4, 4, 4)])
def test_gauge_transformed_abelian_field_is_recovered(extent):
    """U^Omega_{x,mu} = Omega_x U_{x,mu} Omega_{x+mu}^dagger with Omega close
    to 1: the reduction reaches R = 1 (an Abelian field again), and its
    plaquette angles equal the original ones modulo 2 pi."""
    d, V = len(extent), int(np.prod(extent))
    phi = GI.orbit_angles(extent, 7, 2)
    U = abelian_links(phi)
    rng = np.random.default_rng(5)
    a = 0.2 * rng.normal(size=(V, 3))
    t = np.linalg.norm(a, axis=1)
    Om = np.column_stack([np.cos(t), np.sin(t)[:, None] * a / t[:, None]])
    fwd, _ = O.neighbours(extent)
    Ut = np.stack([O.q_mul(O.q_mul(Om, U[mu]), O.q_conj(Om[fwd[mu]])) for mu in range(d)])
    out, sweeps, R, conv = O.mag_project(extent, Ut, eps=1e-26)
    assert conv and sweeps > 1
    assert R > 1.0 - 1e-12
    dp = plaquette_angles(extent, out) - plaquette_angles(extent, phi)
    assert np.max(np.abs(np.angle(np.exp(1j * dp)))) < 1e-9


def test_functional_never_decreases_and_ends_at_a_local_maximum():
    extent = (4, 4, 4)
    d, V = 3, 64
    U = GI.su2_links(extent, 0, 0)
    Rs = [O.mag_project(extent, U, eps=0.0, max_sweeps=k)[2] for k in range(1, 9)]
    assert all(b >= a - 1e-15 for a, b in zip(Rs, Rs[1:]))
    phi, sweeps, R, conv, g = O.mag_project(extent, U, want_g=True)
    assert conv
    rng = np.random.default_rng(9)
    for _ in range(20):
        x = int(rng.integers(V))
        v = 1e-3 * rng.normal(size=3)
        t = np.linalg.norm(v)
        e = np.concatenate([[math.cos(t)], math.sin(t) * v / t])
        g2 = g.copy()
        g2[x] = O.q_mul(e, g[x])
        R2 = float(O.q_rot3(O.mag_transformed(extent, U, g2))[..., 2].sum()) / (d * V)
        assert R2 <= R + 1e-15
