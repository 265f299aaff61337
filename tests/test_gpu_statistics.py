"""GPU: orbit statistics at lattice sizes the oracle cannot sample in seconds.

Fresh beta = 0 orbits (the paper's own are not published), enumerated in
batches of many orbits per launch with plain relaxation (omega = 1, as in the
paper), must reproduce the orbit averages the paper prints: x = F/(dV) at the
global minimum (Tab. III) and, where the paper's curves had reached their
plateau (6x6), the number of distinct minima (Tab. I).  The bound is three
combined standard errors of the two orbit samples, as in the oracle's own
check of the same tables at the small sizes."""
import math
import os
import sys

import numpy as np
import pytest

import gribov_inputs as GI
import paper_1403_0555_amd as gc
from oracle import oracle as O

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ORBIT_SEED = 11


def note(msg):
    print("[gpu-statistics] " + msg, flush=True)
    sys.stdout.flush()


def _paper_row(extent, table):
    name = "x".join(str(n) for n in extent)
    with open(os.path.join(GOLD, "paper_tables.txt")) as f:
        for ln in f:
            w = ln.split()
            if w and not ln.startswith("#") and w[0] == name and w[1] == table:
                return int(w[2]), float(w[3]), float(w[4])
    raise KeyError((extent, table))


def _orbit_sample(extent, n_orbits, n_starts, per_launch):
    """Distinct copies and x at the global minimum for orbits 0..n_orbits-1."""
    counts, gmin = [], []
    params = gc.SolveParams(omega=1.0)
    with gc.Context(0) as ctx:
        for first in range(0, n_orbits, per_launch):
            idx = range(first, min(n_orbits, first + per_launch))
            hs = [ctx.gc_orbit_random(extent, ORBIT_SEED, oi) for oi in idx]
            ctx.gc_launch_batch(hs, [n_starts] * len(hs), params)
            for h in hs:
                assert ctx.gc_wait(h) == gc.GC_OK
                c = ctx.gc_fetch(h)
                assert int(c["hits"].sum()) == n_starts
                counts.append(len(c))
                gmin.append(float(c["x"].min()))
                ctx.gc_release(h)
    return np.array(counts, float), np.array(gmin)


def _agrees(ours, row):
    n, mean, sd = row
    se = math.sqrt(sd ** 2 / n + ours.std() ** 2 / len(ours))
    return abs(ours.mean() - mean) < 3 * se, (ours.mean(), ours.std(), mean, sd, 3 * se)


@pytest.mark.parametrize("extent,n_starts,per_launch", [
    ((6, 6), 1 << 18, 50), ((8, 8), 1 << 18, 50), ((10, 10), 1 << 18, 25),
    ((6, 6, 6), 1 << 18, 25), ((8, 8, 8), 1 << 18, 10), ((4, 4, 4, 4), 1 << 18, 7)])
def test_global_minimum_matches_table_iii(extent, n_starts, per_launch):
    row = _paper_row(extent, "III")
    note(f"Tab. III {extent}: {row[0]} orbits x {n_starts} starts")
    _, gmin = _orbit_sample(extent, row[0], n_starts, per_launch)
    ok, info = _agrees(gmin, row)
    note(f"  ours {info[0]:.4f} +- {info[1]:.4f}, paper {info[2]} +- {info[3]}, bound {info[4]:.4f}")
    assert ok, info
    assert np.all(gmin > 0) and np.all(gmin < 1)


def test_distinct_minima_match_table_i_at_plateau():
    extent = (6, 6)
    row = _paper_row(extent, "I")
    note(f"Tab. I {extent}: {row[0]} orbits x 2^20 starts")
    counts, _ = _orbit_sample(extent, row[0], 1 << 20, 20)
    ok, info = _agrees(counts, row)
    note(f"  ours {info[0]:.1f} +- {info[1]:.1f}, paper {info[2]} +- {info[3]}, bound {info[4]:.1f}")
    assert ok, info


# ---------------------------------------------------------------------------
# Distributions of the minima (Sec. IV.B) computed on the device
# ---------------------------------------------------------------------------

def _copy_dicts(c):
    return [dict(F=float(r["F"]), flags=int(r["flags"]), hits=int(r["hits"])) for r in c]


HIST_CASES = [(gc.GC_HIST_X, gc.GC_HIST_COPIES, 0, 0.0, 0.5, 50),
              (gc.GC_HIST_X, gc.GC_HIST_STARTS, gc.GC_FLAG_IN_REGION, 0.1, 0.4, 300),
              (gc.GC_HIST_REL, gc.GC_HIST_COPIES, gc.GC_FLAG_IN_REGION, 0.0, 0.6, 60),
              (gc.GC_HIST_REL, gc.GC_HIST_STARTS, 0, 0.01, 0.3, 7)]


@pytest.mark.parametrize("extent,n_orbits,n_starts", [((4, 4), 120, 3000), ((6, 6), 100, 20000),
                                                      ((4, 4, 4), 100, 20000)])
def test_histograms_of_many_orbits(extent, n_orbits, n_starts):
    """gc_histogram over >= 100 orbits of one batch equals the oracle's
    histogram definition applied to each orbit's fetched copies (same values,
    same bins: exact counts), and on the smallest lattice equals it applied to
    the oracle's own copy tables of the same orbits."""
    note(f"histograms {extent}: {n_orbits} orbits x {n_starts} starts")
    d, V = len(extent), int(np.prod(extent))
    params = gc.SolveParams(omega=1.0)
    with gc.Context(0) as ctx:
        hs = [ctx.gc_orbit_random(extent, ORBIT_SEED, oi) for oi in range(n_orbits)]
        ctx.gc_launch_batch(hs, [n_starts] * n_orbits, params)
        for h in hs:
            assert ctx.gc_wait(h) == gc.GC_OK
        fetched = [_copy_dicts(ctx.gc_fetch(h)) for h in hs]
        for q, w, req, lo, hi, nb in HIST_CASES:
            got = ctx.gc_histogram(hs, lo, hi, nb, quantity=q, weight=w, require_flags=req)
            want = np.stack([O.histogram(c, d, V, q, w, req, lo, hi, nb) for c in fetched])
            assert np.array_equal(got, want), (q, w, req)
            n_counted = [sum((e["flags"] & req) == req for e in c) for c in fetched]
            if w == gc.GC_HIST_COPIES:
                assert np.array_equal(got.sum(axis=1), n_counted)
        if extent == (4, 4):
            # the oracle's own tables: same copies, F within 1e-10 per site, so
            # a count may move only where a value lies that close to a bin edge
            for oi in range(10):
                phi = GI.orbit_angles(extent, ORBIT_SEED, oi)
                tab = O.enumerate_copies(extent, phi, np.arange(n_starts),
                                         O.SolveParams(omega=1.0, orbit_index=oi))["table"]
                for q, w, req, lo, hi, nb in HIST_CASES:
                    want = O.histogram(tab.values(), d, V, q, w, req, lo, hi, nb)
                    got = ctx.gc_histogram([hs[oi]], lo, hi, nb, quantity=q, weight=w, require_flags=req)[0]
                    if not np.array_equal(got, want):
                        width = (hi - lo) / nb
                        Fg = min(e["F"] for e in tab.values() if (e["flags"] & req) == req)
                        vals = [e["F"] / (d * V) if q == gc.GC_HIST_X else (e["F"] - Fg) / Fg
                                for e in tab.values()]
                        near = [v for v in vals if abs((v - lo) / width - round((v - lo) / width)) < 1e-8]
                        assert near, (oi, q, w, got, want)
        # errors
        with pytest.raises(gc.GcError):
            ctx.gc_histogram(hs[:1], 1.0, 0.0, 10)
        h_new = ctx.gc_orbit_random(extent, ORBIT_SEED, 999)
        with pytest.raises(gc.GcError) as e:
            ctx.gc_histogram([h_new], 0.0, 1.0, 10)
        assert e.value.status == gc.GC_ESTATE
