"""GPU: relaxation from the caller's gauge transformations (gc_launch_from).

* Hot orbits: random caller angles relax to the same copies as the oracle
  started from the same angles (keys, hits, F, lambda2, flags).
* The trivial orbit (Sec. I; all links 1): the twisted states
  theta_x = sum_mu 2 pi k_mu x_mu / N_mu are stationary with uniform link
  angles a_mu = 2 pi k_mu / N_mu, so F = V sum_mu (1 - cos a_mu), and the
  Faddeev-Popov operator is sum_mu cos a_mu times the lattice Laplacian along
  mu.  Its lowest non-constant eigenvalue is
    min_mu 2 cos a_mu (1 - cos(2 pi / N_mu))      when every cos a_mu > 0,
    0 (a singular state, Sec. II)                   when min cos a_mu = 0,
    min_mu 4 cos a_mu (a saddle)                    when some cos a_mu < 0,
  the last for even extents, where the momentum pi exists.  Each state is
  classified after its first sweep without moving.
"""
import math
import sys

import numpy as np
import pytest

import gribov_inputs as GI
import paper_1403_0555_amd as gc
from oracle import oracle as O

pytestmark = pytest.mark.gpu

TWO_PI = 2.0 * math.pi
F_TOL_PER_SITE = 1e-10
LAMBDA_TOL = 1e-8


def note(msg):
    print("[gpu-states] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gc.Context(0)
    yield c
    c.close()


def twisted(extent, k):
    d = len(extent)
    V = int(np.prod(extent))
    coords = np.array(np.unravel_index(np.arange(V), extent[::-1]))[::-1]
    return sum(TWO_PI * k[mu] * coords[mu] / extent[mu] for mu in range(d))


def expected(extent, k):
    V = int(np.prod(extent))
    a = [TWO_PI * k[mu] / extent[mu] for mu in range(len(extent))]
    F = V * sum(1 - math.cos(x) for x in a)
    c = [math.cos(x) for x in a]
    if min(c) > 1e-12:
        lam = min(2 * c[mu] * (1 - math.cos(TWO_PI / extent[mu])) for mu in range(len(extent)))
        flag = gc.GC_FLAG_IN_REGION
    elif min(c) > -1e-12:
        lam, flag = 0.0, gc.GC_FLAG_SINGULAR
    else:
        lam, flag = 4 * min(c), gc.GC_FLAG_SADDLE
    return F, lam, flag


CASES = [
    ((8, 8), [(0, 0), (1, 0), (0, -1), (1, 1), (-1, 1), (2, 0), (2, 1), (3, 0), (0, 3)]),
    ((6, 6, 6), [(0, 0, 0), (1, 0, -1), (1, 1, 1), (0, 0, 1)]),
    ((4, 4, 4, 4), [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 1)]),
    ((6, 6, 6, 6), [(0, 0, 0, 0), (1, 0, 0, 0), (1, -1, 1, -1)]),
]


@pytest.mark.parametrize("extent,ks", CASES)
@pytest.mark.parametrize("omega", [1.0, 1.7])
def test_twisted_states_of_the_trivial_orbit(ctx, extent, ks, omega):
    note(f"twisted states {extent} omega={omega}: {len(ks)} states")
    theta = np.stack([twisted(extent, k) for k in ks])
    h = ctx.gc_orbit_load(extent, GI.cold_orbit(extent))
    ctx.gc_launch_from(h, theta, gc.SolveParams(omega=omega))
    assert ctx.gc_wait(h, 120_000) == gc.GC_OK
    starts = ctx.gc_fetch_starts(h, len(ks))
    copies = ctx.gc_fetch(h)
    V = int(np.prod(extent))
    assert len(copies) == len(ks)                # distinct windings, distinct keys
    by_rep = {int(c["rep_start"]): c for c in copies}
    for s, k in enumerate(ks):
        F, lam, flag = expected(extent, k)
        r = starts[s]
        assert r["status"] == gc.GC_START_CONVERGED
        assert abs(r["F"] - F) / V < F_TOL_PER_SITE, (k, r["F"], F)
        # the oracle's key of the same state
        o_rec, _, _, _ = O.observe(extent, GI.cold_orbit(extent), theta[s])
        assert (int(r["key_hi"]), int(r["key_lo"])) == (int(o_rec["key_hi"]), int(o_rec["key_lo"]))
        c = by_rep[s]
        assert int(c["hits"]) == 1 and int(c["first_start"]) == s
        assert abs(c["lambda2"] - lam) < LAMBDA_TOL, (k, c["lambda2"], lam)
        assert (int(c["flags"]) & 7) == flag, (k, int(c["flags"]), flag)
        # it did not move: the stored state is the given one up to a global phase
        t = ctx.gc_fetch_start_state(h, s)
        dt = np.angle(np.exp(1j * (t - (theta[s] - theta[s][-1]))))
        assert np.max(np.abs(dt)) < 1e-9
    ctx.gc_release(h)


@pytest.mark.parametrize("extent,n,prec", [((6, 6), 300, "fp64"), ((4, 4, 4, 4), 200, "fp64"),
                                            ((8, 8, 8), 100, "mixed")])
def test_caller_starts_match_oracle(ctx, extent, n, prec):
    """Hot orbit, caller angles drawn uniformly: the GPU relaxes them exactly
    as the oracle does from the same angles."""
    V = int(np.prod(extent))
    phi = GI.orbit_angles(extent, 5, 3)
    theta = (GI.uniform01(9, (0, 0, 0, 0x54), n * V).reshape(n, V) * TWO_PI) - math.pi
    p = gc.SolveParams(omega=1.7, precision=prec)
    note(f"caller starts {extent} n={n} {prec}")
    h = ctx.gc_orbit_load(extent, phi)
    ctx.gc_launch_from(h, theta, p)
    assert ctx.gc_wait(h, 300_000) == gc.GC_OK
    starts = ctx.gc_fetch_starts(h, n)
    copies = ctx.gc_fetch(h)
    op = O.SolveParams(omega=1.7, precision=prec)
    rec, _, _ = O.solve(extent, phi, np.arange(n), op, theta_init=theta)
    conv = rec["status"] == O.CONVERGED
    same = (starts["key_hi"] == rec["key_hi"]) & (starts["key_lo"] == rec["key_lo"])
    if prec == "fp64":
        assert np.array_equal(starts["status"], rec["status"])
        assert np.all(same[conv])
        assert np.max(np.abs(starts["F"][conv] - rec["F"][conv])) / V < F_TOL_PER_SITE
    else:
        # FP32 bulk: a start near a basin boundary may take the other basin
        assert np.mean(same[conv]) >= 0.97
    # every copy's representative is a start that reached its key
    for c in copies:
        r = int(c["rep_start"])
        assert (starts["key_hi"][r], starts["key_lo"][r]) == (c["key_hi"], c["key_lo"])
    assert int(copies["hits"].sum()) == int(np.sum(starts["status"] == gc.GC_START_CONVERGED))
    ctx.gc_release(h)


def test_launch_from_rejects_bad_angles(ctx):
    h = ctx.gc_orbit_load((4, 4), GI.cold_orbit((4, 4)))
    bad = np.zeros((2, 16))
    bad[1, 3] = np.nan
    with pytest.raises(gc.GcError) as e:
        ctx.gc_launch_from(h, bad)
    assert e.value.status == gc.GC_EINVAL
    ctx.gc_release(h)
