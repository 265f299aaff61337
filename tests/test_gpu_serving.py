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
    """Tuned kernel variants compute the same copies bit for bit: the
    variants differ in where coefficients live, not in the arithmetic or its
    order."""
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
        assert r["relax_variant"] in (0, 1, 2)
        assert r["post_block"] * r["post_sites_per_thread"] >= V
        assert r["relax_ms"] > 0 and r["post_ms"] > 0
        ctx.gc_launch(h, n, params)
        assert ctx.gc_wait(h) == gc.GC_OK
        got = ctx.gc_fetch(h)
        for f in ("key_hi", "key_lo", "hits", "first_start", "rep_start", "flags", "F", "lambda2",
                  "lanczos_iters"):
            assert np.array_equal(got[f], ref[f]), f
        ctx.gc_release(h)


def _oracle_params(p, oi):
    from oracle import oracle as O
    return O.SolveParams(omega=p.omega, precision="fp64", eps64=p.eps64, start_seed=p.start_seed, orbit_index=oi)


def test_served_mix_matches_oracle():
    """Requests admitted while others run (mixed precision, including the 8^4
    lattice with 10^4 starts, the largest request of the serving workload):
    every served orbit against the double-precision oracle on sampled
    starts.  Keys agree on every start whose basin the single-precision bulk
    did not move (at most 1 % of the sample), F within 1e-10 per site there,
    and every other sampled start is a genuine double-precision minimum."""
    from oracle import bruteforce as BF
    from oracle import oracle as O
    p = gc.SolveParams(omega=1.7, precision="mixed")
    mix = [((8, 8, 8, 8), 10_000, 11), ((6, 6, 6, 6), 4000, 12), ((8, 8, 8), 6000, 13), ((16, 16), 5000, 14),
           ((4, 4, 4, 4), 8000, 15), ((10, 10), 3000, 16)]
    with gc.Context(0, n_streams=4) as ctx:
        hs = []
        for ext, n, oi in mix:
            phi = GI.orbit_angles(ext, 0, oi)
            h = ctx.gc_orbit_load(ext, phi, oi)
            ctx.gc_launch(h, n, p)
            hs.append((h, ext, n, oi, phi))
        for h, ext, n, oi, phi in hs:
            assert ctx.gc_wait(h, 600_000) == gc.GC_OK
            copies, starts = ctx.gc_fetch(h), ctx.gc_fetch_starts(h, n)
            V = int(np.prod(ext))
            assert int(copies["hits"].sum()) == n == int(np.sum(starts["status"] == gc.GC_START_CONVERGED))
            k = [(int(a), int(b)) for a, b in zip(copies["key_hi"], copies["key_lo"])]
            assert all(x < y for x, y in zip(k, k[1:]))
            m = 24 if V >= 4096 else 120
            ids = np.unique(np.linspace(0, n - 1, m).astype(np.int64))
            note("served %s n=%d: oracle on %d sampled starts" % (ext, n, ids.size))
            rec, _, _ = O.solve(ext, phi, ids, _oracle_params(p, oi))
            gs = starts[ids]
            same = (gs["key_hi"] == rec["key_hi"]) & (gs["key_lo"] == rec["key_lo"])
            assert np.sum(~same) <= max(1, int(0.01 * ids.size)), int(np.sum(~same))
            assert np.max(np.abs(gs["F"][same] - rec["F"][same])) / V < 1e-10
            land = BF.Landscape(ext, phi)
            for s in ids[~same]:
                th = ctx.gc_fetch_start_state(h, int(s))
                assert np.mean(land.grad(th) ** 2) < 2e-14
            ctx.gc_release(h)


def test_launch_does_not_block_while_jobs_run():
    """gc_launch only enqueues: with more launches in flight than streams it
    returns at once (queued launches start as streams free up)."""
    import time
    ext, n = (6, 6, 6, 6), 20_000
    p = gc.SolveParams(omega=1.7, precision="mixed")
    phi = GI.orbit_angles(ext, 0, 0)
    with gc.Context(0, n_streams=4) as ctx:
        hs = [ctx.gc_orbit_load(ext, phi, 0) for _ in range(8)]
        # warm-up: code objects loaded, pools filled
        for h in hs[:4]:
            ctx.gc_launch(h, n, p)
        for h in hs[:4]:
            assert ctx.gc_wait(h) == gc.GC_OK
        times = []
        for h in hs:
            t0 = time.perf_counter()
            ctx.gc_launch(h, n, p)
            times.append((time.perf_counter() - t0) * 1e3)
        running = sum(ctx.gc_poll(h)["state"] in (gc.GC_ORBIT_RUNNING, gc.GC_ORBIT_QUEUED) for h in hs)
        note("gc_launch ms: %s; %d in flight" % (["%.2f" % t for t in times], running))
        assert running >= 5
        assert max(times) < 20.0
        # polls and the release of a finished orbit while others still run stay fast
        assert ctx.gc_wait(hs[0]) == gc.GC_OK
        t0 = time.perf_counter()
        ctx.gc_poll(hs[1])
        ctx.gc_release(hs[0])
        assert (time.perf_counter() - t0) * 1e3 < 50.0
        for h in hs[1:]:
            assert ctx.gc_wait(h) == gc.GC_OK
            ctx.gc_release(h)


def test_budget_is_a_hard_limit():
    """Unreleased results count against the budget: a launch that does not
    fit waits; with nothing running gc_wait reports GC_ENOMEM instead of
    blocking; releasing the earlier results lets it run."""
    ext, n = (4, 4, 4, 4), 4000
    params = gc.SolveParams(omega=1.0)
    with gc.Context(0) as probe:
        h = probe.gc_orbit_load(ext, GI.orbit_angles(ext, 0, 0), 0)
        need = probe.gc_launch_bytes(h, n, params)
    with gc.Context(0, hbm_budget_bytes=int(need * 1.5)) as ctx:
        h1 = ctx.gc_orbit_load(ext, GI.orbit_angles(ext, 0, 0), 0)
        h2 = ctx.gc_orbit_load(ext, GI.orbit_angles(ext, 0, 0), 0)
        ctx.gc_launch(h1, n, params)
        assert ctx.gc_wait(h1) == gc.GC_OK
        ref = _results(ctx, h1, n)
        ctx.gc_launch(h2, n, params)
        assert ctx.gc_poll(h2)["state"] == gc.GC_ORBIT_QUEUED
        info = ctx.gc_memory_info()
        assert info["in_use"] <= info["budget"] and info["queued"] == 1
        with pytest.raises(gc.GcError) as e:
            ctx.gc_wait(h2, 10_000)
        assert e.value.status == gc.GC_ENOMEM
        ctx.gc_release(h1)
        assert ctx.gc_wait(h2, 120_000) == gc.GC_OK
        _same(_results(ctx, h2, n), ref)
        ctx.gc_release(h2)


def test_launches_on_the_callers_stream():
    """With a caller stream every launch is enqueued on it, after the
    caller's earlier work: the stream is busy while the launch runs and a
    synchronisation of the stream finishes the launch.  The stream comes from
    the HIP runtime the library links (PyTorch in this image bundles another
    HIP runtime, which cannot share a process with it)."""
    import ctypes
    gc.lib()
    hip = ctypes.CDLL("libamdhip64.so.7")
    stream, buf = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipStreamCreateWithFlags(ctypes.byref(stream), 1) == 0
    assert hip.hipMalloc(ctypes.byref(buf), ctypes.c_size_t(1 << 30)) == 0
    ext, n = (6, 6, 6, 6), 50_000
    phi = GI.orbit_angles(ext, 0, 0)
    p = gc.SolveParams(omega=1.7)
    try:
        with gc.Context(0) as ref_ctx:
            h = ref_ctx.gc_orbit_load(ext, phi, 0)
            ref_ctx.gc_launch(h, 2000, p)
            assert ref_ctx.gc_wait(h) == gc.GC_OK
            ref = _results(ref_ctx, h, 2000)
        with gc.Context(0, hip_stream=stream.value) as ctx:
            h = ctx.gc_orbit_load(ext, phi, 0)
            assert hip.hipStreamSynchronize(stream) == 0
            ctx.gc_launch(h, n, p)
            assert hip.hipStreamQuery(stream) != 0          # busy with the launch alone
            assert hip.hipStreamSynchronize(stream) == 0
            assert ctx.gc_wait(h, 5000) == gc.GC_OK
            # caller work first, then the launch behind it on the same stream
            for _ in range(16):
                assert hip.hipMemsetAsync(buf, 0, ctypes.c_size_t(1 << 30), stream) == 0
            ctx.gc_launch(h, 2000, p)
            assert hip.hipStreamSynchronize(stream) == 0
            assert ctx.gc_wait(h, 5000) == gc.GC_OK
            _same(_results(ctx, h, 2000), ref)
            ctx.gc_release(h)
    finally:
        hip.hipFree(buf)
        hip.hipStreamDestroy(stream)
