"""GPU: continuous batching and admission.

Launches that arrive while others run are admitted as HBM frees up and their
work overlaps on the device; every orbit's result must be the same alone and
in the mix (here bit-identical: per-start arithmetic does not depend on
co-scheduling), and a launch larger than the budget is refused."""
import sys

import numpy as np
import pytest

import gribov_inputs as GI
import paper_1403_0555_amd as gc

pytestmark = pytest.mark.gpu

SHAPES = [((4, 4, 4, 4), 3000, 0), ((8, 8, 8), 2000, 1), ((6, 6, 6, 6), 600, 2), ((12, 12), 4000, 3),
          ((3, 3), 500, 4)]


def note(msg):
    print("[gpu-serving] " + msg, flush=True)
    sys.stdout.flush()


def _results(ctx, h, n):
    return ctx.gc_fetch(h), ctx.gc_fetch_starts(h, n)


def _same_fields(x, y):
    assert x.shape == y.shape
    for name in x.dtype.names:
        fx, fy = x[name], y[name]
        nan_ok = fx.dtype.kind == "f"
        assert np.array_equal(fx, fy, equal_nan=nan_ok), name


def _same(a, b):
    ca, sa = a
    cb, sb = b
    _same_fields(ca, cb)
    _same_fields(sa, sb)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_alone_equals_mix(precision):
    params = gc.SolveParams(omega=1.7, precision=precision)
    with gc.Context(0) as ctx:
        alone = {}
        for ext, n, oi in SHAPES:
            note("alone %s n=%d %s" % (ext, n, precision))
            h = ctx.gc_orbit_load(ext, GI.orbit_angles(ext, 5, oi), oi)
            ctx.gc_launch(h, n, params)
            assert ctx.gc_wait(h) == gc.GC_OK
            alone[oi] = _results(ctx, h, n)
            ctx.gc_release(h)
        note("mix")
        hs = []
        for ext, n, oi in SHAPES:
            h = ctx.gc_orbit_load(ext, GI.orbit_angles(ext, 5, oi), oi)
            ctx.gc_launch(h, n, params)
            hs.append((h, n, oi))
        for h, n, oi in hs:
            assert ctx.gc_wait(h) == gc.GC_OK
            _same(_results(ctx, h, n), alone[oi])
            ctx.gc_release(h)
        note("batch")
        hs = []
        for ext, n, oi in SHAPES:
            hs.append((ctx.gc_orbit_load(ext, GI.orbit_angles(ext, 5, oi), oi), n, oi))
        ctx.gc_launch_batch([h for h, _, _ in hs], [n for _, n, _ in hs], params)
        for h, n, oi in hs:
            assert ctx.gc_wait(h) == gc.GC_OK
            _same(_results(ctx, h, n), alone[oi])
            ctx.gc_release(h)


def test_budget_admission_queues_then_runs():
    ext, n = (4, 4, 4, 4), 4000
    params = gc.SolveParams(omega=1.0)
    with gc.Context(0) as probe:
        h = probe.gc_orbit_load(ext, GI.orbit_angles(ext, 0, 0), 0)
        need = probe.gc_launch_bytes(h, n, params)
        probe.gc_launch(h, n, params)
        probe.gc_wait(h)
        ref = _results(probe, h, n)
    with gc.Context(0, hbm_budget_bytes=int(need * 1.5)) as ctx:
        h1 = ctx.gc_orbit_load(ext, GI.orbit_angles(ext, 0, 0), 0)
        h2 = ctx.gc_orbit_load(ext, GI.orbit_angles(ext, 0, 0), 0)
        ctx.gc_launch(h1, n, params)
        ctx.gc_launch(h2, n, params)
        info = ctx.gc_memory_info()
        assert info["in_use"] <= info["budget"]
        st2 = ctx.gc_poll(h2)["state"]
        assert st2 in (gc.GC_ORBIT_QUEUED, gc.GC_ORBIT_DONE)
        assert ctx.gc_wait(h1) == gc.GC_OK
        _same(_results(ctx, h1, n), ref)
        ctx.gc_release(h1)            # frees the budget for the queued launch
        assert ctx.gc_wait(h2, 120_000) == gc.GC_OK
        _same(_results(ctx, h2, n), ref)
        # larger than the whole budget: refused
        with pytest.raises(gc.GcError) as e:
            ctx.gc_launch(h2, 10 * n, params)
        assert e.value.status == gc.GC_ENOMEM
        ctx.gc_release(h2)


def test_launch_while_busy_is_refused():
    ext = (6, 6, 6, 6)
    with gc.Context(0) as ctx:
        h = ctx.gc_orbit_load(ext, GI.orbit_angles(ext, 0, 0), 0)
        ctx.gc_launch(h, 20000, gc.SolveParams(omega=1.7))
        if ctx.gc_poll(h)["state"] != gc.GC_ORBIT_DONE:
            with pytest.raises(gc.GcError) as e:
                ctx.gc_launch(h, 10)
            assert e.value.status == gc.GC_EBUSY
        assert ctx.gc_wait(h) == gc.GC_OK
        ctx.gc_release(h)


@pytest.mark.parametrize("extent,precision,n", [((4, 4, 4, 4), "fp64", 3000), ((8, 8, 8), "mixed", 2000)])
def test_autotune_keeps_results(extent, precision, n):
    """Tuned kernel variants compute the same copies: keys, hits and first
    starts identical, F and lambda2 within rounding of a different
    reduction order."""
    params = gc.SolveParams(omega=1.7 if precision == "mixed" else 1.0, precision=precision)
    phi = GI.orbit_angles(extent, 2, 9)
    V = int(np.prod(extent))
    with gc.Context(0) as ctx:
        h = ctx.gc_orbit_load(extent, phi, 9)
        ctx.gc_launch(h, n, params)
        assert ctx.gc_wait(h) == gc.GC_OK
        ref = ctx.gc_fetch(h)
        note("autotune %s %s" % (extent, precision))
        r = ctx.gc_autotune(h, n, params)
        assert r["relax_variant"] % 8 in (0, 1, 2) and r["relax_variant"] in (0, 1, 2, 8, 9, 10)
        assert r["post_block"] * r["post_sites_per_thread"] >= V
        assert r["relax_ms"] > 0 and r["post_ms"] > 0
        ctx.gc_launch(h, n, params)
        assert ctx.gc_wait(h) == gc.GC_OK
        got = ctx.gc_fetch(h)
        for f in ("key_hi", "key_lo", "hits", "first_start"):
            assert np.array_equal(got[f], ref[f]), f
        assert np.max(np.abs(got["F"] - ref["F"])) / V < 1e-12
        assert np.max(np.abs(got["lambda2"] - ref["lambda2"])) < 1e-10
        ctx.gc_release(h)
