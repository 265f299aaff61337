"""GPU parity: the HIP path against the oracle on the same seeded inputs.

Bar (per start, FP64 mode): identical status and integer key (bit-exact),
sweep counts equal (a stop decision taken within rounding of the threshold
may move by one sweep), functional F within 1e-10 per site, and the copy table
identical (keys, hits, lowest start id).  lambda2 of each copy (Lanczos on
the GPU, dense LAPACK in the oracle, both from the copy's lowest start) within
1e-8.  Mixed mode: keys bit-identical wherever the single-precision
trajectory reaches the same minimum as the double one; every other start's
copy is checked to be a genuine double-precision minimum.
"""
import math
import sys

import numpy as np
import pytest

import gribov_inputs as GI
import paper_1403_0555_amd as gc
from oracle import bruteforce as BF
from oracle import oracle as O

pytestmark = pytest.mark.gpu

F_TOL_PER_SITE = 1e-10
LAMBDA_TOL = 1e-8


def note(msg):
    print("[gpu-parity] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gc.Context(0)
    yield c
    c.close()


def run_gpu(ctx, extent, phi, n, params, orbit_index=0):
    note("launch extent=%s n=%d omega=%s prec=%s" % (extent, n, params.omega, params.precision))
    h = ctx.gc_orbit_load(extent, phi, orbit_index)
    ctx.gc_launch(h, n, params)
    assert ctx.gc_wait(h, 600_000) == gc.GC_OK
    copies = ctx.gc_fetch(h)
    starts = ctx.gc_fetch_starts(h, n)
    prog = ctx.gc_poll(h)
    return h, copies, starts, prog


def oracle_params(p: gc.SolveParams, orbit_index=0) -> O.SolveParams:
    return O.SolveParams(omega=p.omega, precision=p.precision, eps32=p.eps32, eps64=p.eps64,
                         stop_norm=p.stop_norm, check_every=p.check_every, max_sweeps=p.max_sweeps,
                         start_seed=p.start_seed, orbit_index=orbit_index)


def compare_starts(extent, g, o, allow_sweep_slack=1):
    V = int(np.prod(extent))
    assert np.array_equal(g["status"], o["status"])
    conv = o["status"] == O.CONVERGED
    assert np.array_equal(g["key_hi"][conv], o["key_hi"][conv])
    assert np.array_equal(g["key_lo"][conv], o["key_lo"][conv])
    dsw = np.abs(g["sweeps64"].astype(np.int64) - o["sweeps64"])
    assert dsw.max() <= allow_sweep_slack
    assert np.mean(dsw == 0) > 0.99
    if conv.any():
        assert np.max(np.abs(g["F"][conv] - o["F"][conv])) / V < F_TOL_PER_SITE
        assert np.array_equal(g["paper_X"][conv], o["paper_X"][conv]) or \
            np.max(np.abs(g["paper_X"][conv].astype(np.int64) - o["paper_X"][conv])) <= 1


def assert_key_order(copies):
    """gc_fetch returns the copies in strictly increasing (key_hi, key_lo)."""
    k = [(int(a), int(b)) for a, b in zip(copies["key_hi"], copies["key_lo"])]
    assert all(x < y for x, y in zip(k, k[1:]))


def compare_tables(extent, phi, copies, o_res, params, check_lambda=True):
    V = int(np.prod(extent))
    tab = o_res["table"]
    assert_key_order(copies)
    gk = {(int(c["key_hi"]), int(c["key_lo"])): c for c in copies}
    assert set(gk) == set(tab)
    for k, e in tab.items():
        c = gk[k]
        assert int(c["hits"]) == e["hits"]
        assert int(c["first_start"]) == e["first_start"]
        assert int(c["rep_start"]) == e["rep_start"]
        assert abs(c["F"] - e["F"]) / V < F_TOL_PER_SITE
        assert (int(c["flags"]) & gc.GC_FLAG_COLLISION) == (e["flags"] & O.FLAG_COLLISION)
        if check_lambda:
            assert abs(c["lambda2"] - e["lambda2"]) < LAMBDA_TOL, (c["lambda2"], e["lambda2"])
            assert (int(c["flags"]) & 7) == (e["flags"] & 7)


def check_start_filter(copies, starts, o_res, first_start=0):
    """The filter's result sits in the start record of each copy's
    representative (the same bits as the copy) and nowhere else."""
    gk = {(int(c["key_hi"]), int(c["key_lo"])): c for c in copies}
    reps = set()
    for k, e in o_res["table"].items():
        r = e["rep_start"] - first_start
        reps.add(r)
        c = gk[k]
        assert starts["lambda2"][r] == c["lambda2"]
        assert starts["lanczos_iters"][r] == c["lanczos_iters"]
        assert (int(starts["flags"][r]) & 7) == (int(c["flags"]) & 7)
    others = np.ones(len(starts), bool)
    others[list(reps)] = False
    assert np.all(np.isnan(starts["lambda2"][others]))
    assert np.all(starts["lanczos_iters"][others] == 0)
    assert np.all((starts["flags"][others] & 7) == 0)


# ---------------------------------------------------------------------------

def test_orbit_random_matches_input_generator(ctx):
    for extent, seed, oi in [((4, 4), 0, 0), ((6, 6, 6, 6), 3, 7), ((10, 10, 10), 0, 2)]:
        h = ctx.gc_orbit_random(extent, seed, oi)
        assert np.array_equal(ctx.gc_orbit_angles(h), GI.orbit_angles(extent, seed, oi))
        ctx.gc_release(h)


def test_small_2d_workload_full_parity(ctx):
    """2D 4x4, 1000 starts, omega 1.7, FP64, filter on: every start and the table."""
    extent = (4, 4)
    phi = GI.orbit_angles(extent, 0, 0)
    p = gc.SolveParams(omega=1.7)
    h, copies, starts, prog = run_gpu(ctx, extent, phi, 1000, p)
    o = O.enumerate_copies(extent, phi, np.arange(1000), oracle_params(p))
    compare_starts(extent, starts, o["records"])
    compare_tables(extent, phi, copies, o, p)
    check_start_filter(copies, starts, o)
    assert prog["distinct"] == len(o["table"]) and prog["converged"] == 1000
    assert prog["in_region"] == len(o["table"])
    inreg = copies["flags"] & gc.GC_FLAG_IN_REGION != 0
    assert prog["in_region_hits"] == int(copies["hits"][inreg].sum()) == 1000
    assert prog["lanczos_iters"] == int(copies["lanczos_iters"].sum()) > 0
    # into a caller-owned buffer: the same records, a view of its head
    buf = np.zeros(len(copies) + 5, dtype=gc.COPY_DTYPE)
    again = ctx.gc_fetch(h, out=buf)
    assert again.base is buf and np.array_equal(again, copies)
    with pytest.raises(ValueError):
        ctx.gc_fetch(h, out=np.zeros(len(copies) - 1, dtype=gc.COPY_DTYPE))
    with pytest.raises(ValueError):
        ctx.gc_fetch(h, out=np.zeros(len(copies), dtype=np.float64))
    ctx.gc_release(h)


@pytest.mark.parametrize("extent,omega,n", [
    ((2, 2), 1.7, 300),            # N = 2: forward and backward neighbour coincide
    ((3, 3), 1.0, 300),            # three colours
    ((5, 5), 1.7, 200),            # five colours
    ((7,), 1.0, 400),              # 1D ring, seven colours
    ((8,), 1.0, 400),              # 1D ring, two colours
    ((6, 6), 1.7, 257),            # V = 36: ragged against the block
    ((6, 4, 2), 1.0, 130),
    ((2, 2, 2, 2), 1.7, 300),
    ((4, 4, 4), 1.7, 300),
    ((10, 10, 10), 1.7, 40),       # V = 1000: several site tiles and a ragged tail
    ((6, 6, 6, 6), 1.7, 24),
    ((8, 8, 8), 1.0, 20),
    ((8, 8, 8, 8), 1.7, 3),        # V = 4096: the filter keeps link weights in global memory
])
def test_parity_shapes(ctx, extent, omega, n):
    phi = GI.orbit_angles(extent, 1, 3)
    p = gc.SolveParams(omega=omega)
    h, copies, starts, prog = run_gpu(ctx, extent, phi, n, p, orbit_index=3)
    o = O.enumerate_copies(extent, phi, np.arange(n), oracle_params(p, 3))
    compare_starts(extent, starts, o["records"])
    compare_tables(extent, phi, copies, o, p)
    check_start_filter(copies, starts, o)
    ctx.gc_release(h)


def test_first_start_offset_and_seed(ctx):
    extent = (4, 4, 4)
    phi = GI.orbit_angles(extent, 0, 5)
    p = gc.SolveParams(omega=1.7, first_start=123456789, start_seed=99)
    h, copies, starts, _ = run_gpu(ctx, extent, phi, 100, p, orbit_index=5)
    op = oracle_params(p, 5)
    op.start_seed = 99
    o = O.enumerate_copies(extent, phi, 123456789 + np.arange(100), op)
    compare_starts(extent, starts, o["records"])
    compare_tables(extent, phi, copies, o, p)
    check_start_filter(copies, starts, o, first_start=123456789)
    ctx.gc_release(h)


def test_stopping_variants(ctx):
    extent = (6, 6)
    phi = GI.orbit_angles(extent, 0, 1)
    for p in [gc.SolveParams(omega=1.0, stop_norm="max_abs", eps64=1e-12),
              gc.SolveParams(omega=1.7, check_every=4),
              gc.SolveParams(omega=1.0, max_sweeps=3)]:
        h, copies, starts, _ = run_gpu(ctx, extent, phi, 100, p, orbit_index=1)
        o = O.enumerate_copies(extent, phi, np.arange(100), oracle_params(p, 1))
        compare_starts(extent, starts, o["records"])
        compare_tables(extent, phi, copies, o, p)
        ctx.gc_release(h)


@pytest.mark.parametrize("extent,omega,n", [
    ((10, 10, 10), 1.0, 16),       # 500 sites per colour: eight slots per lane
    ((6, 6, 6, 6), 1.7, 12),       # 648: eleven
])
def test_max_abs_stop_on_exchange_region_kernel(ctx, extent, omega, n):
    """The max |div| stop (the paper's criterion, Sec. III) on lattices of
    the exchange-region kernel (more than two slots per lane), start by
    start and copy by copy against the oracle."""
    phi = GI.orbit_angles(extent, 3, 4)
    p = gc.SolveParams(omega=omega, stop_norm="max_abs", eps64=1e-12)
    h, copies, starts, _ = run_gpu(ctx, extent, phi, n, p, orbit_index=4)
    o = O.enumerate_copies(extent, phi, np.arange(n), oracle_params(p, 4))
    compare_starts(extent, starts, o["records"])
    compare_tables(extent, phi, copies, o, p)
    check_start_filter(copies, starts, o)
    ctx.gc_release(h)


def test_sweep_cap_gives_no_copies(ctx):
    extent = (4, 4)
    phi = GI.orbit_angles(extent, 0, 0)
    h, copies, starts, prog = run_gpu(ctx, extent, phi, 50, gc.SolveParams(max_sweeps=1))
    assert len(copies) == 0
    assert np.all(starts["status"] == gc.GC_START_NONCONVERGED)
    assert prog["nonconverged"] == 50 and prog["distinct"] == 0
    ctx.gc_release(h)


def test_invalid_inputs(ctx):
    extent = (4, 4)
    phi = GI.orbit_angles(extent, 0, 0)
    bad = phi.copy()
    bad[1, 3] = np.nan
    with pytest.raises(gc.GcError) as e:
        ctx.gc_orbit_load(extent, bad)
    assert e.value.status == gc.GC_EINVAL
    with pytest.raises(gc.GcError) as e:
        ctx.gc_orbit_load((3, 5), np.zeros((2, 15)))
    assert e.value.status == gc.GC_EUNSUPPORTED
    h = ctx.gc_orbit_load(extent, phi)
    with pytest.raises(gc.GcError) as e:
        ctx.gc_launch(h, 0)
    assert e.value.status == gc.GC_EINVAL
    with pytest.raises(gc.GcError) as e:
        ctx.gc_launch(h, 10, gc.SolveParams(omega=2.5))
    assert e.value.status == gc.GC_EINVAL
    with pytest.raises(gc.GcError) as e:
        ctx.gc_fetch(h)
    assert e.value.status == gc.GC_ESTATE
    ctx.gc_release(h)


def test_start_state_matches_oracle(ctx):
    """gc_fetch_start_state: theta_i - theta_{V-1} of a start's final state
    equals the oracle's."""
    extent = (4, 4, 4, 4)
    phi = GI.orbit_angles(extent, 0, 0)
    p = gc.SolveParams(omega=1.7)
    h, copies, starts, _ = run_gpu(ctx, extent, phi, 20, p)
    rec, g, _ = O.solve(extent, phi, np.arange(20), oracle_params(p), want_state=True)
    for s in [0, 7, 19]:
        th = ctx.gc_fetch_start_state(h, s)
        ref = O.theta_of(g[s])
        ref = np.angle(np.exp(1j * (ref - ref[-1])))
        d = np.angle(np.exp(1j * (th - ref)))
        assert np.max(np.abs(d)) < 1e-9
        assert th[-1] == 0.0
        # the representative reproduces the copy: same key and F
        r, _, _, _ = O.observe(extent, phi, th)
        assert int(r["key_hi"]) == int(starts["key_hi"][s])
        assert abs(r["F"] - starts["F"][s]) < 1e-10
    ctx.gc_release(h)


# ---------------------------------------------------------------------------
# Full-size workloads: sampled per-start parity + properties at any size
# ---------------------------------------------------------------------------

def V_of(extent):
    return int(np.prod(extent))


def _check_table_properties(extent, copies, starts, prog):
    V = int(np.prod(extent))
    assert_key_order(copies)
    # the representative start reaches its copy's key and carries its F
    rep = copies["rep_start"].astype(np.int64)
    assert np.array_equal(starts["key_hi"][rep], copies["key_hi"])
    assert np.array_equal(starts["key_lo"][rep], copies["key_lo"])
    assert np.array_equal(starts["F"][rep], copies["F"])
    conv = starts["status"] == gc.GC_START_CONVERGED
    keys = set(zip(starts["key_hi"][conv].tolist(), starts["key_lo"][conv].tolist()))
    assert len(keys) == len(copies) == prog["distinct"]
    assert int(copies["hits"].sum()) == int(conv.sum()) == prog["converged"]
    # each copy's lowest start reaches its key; its F is the class's lowest
    first, fmin = {}, {}
    for s in np.nonzero(conv)[0]:
        k = (int(starts["key_hi"][s]), int(starts["key_lo"][s]))
        first.setdefault(k, s)
        fmin[k] = min(fmin.get(k, np.inf), starts["F"][s])
    for c in copies:
        k = (int(c["key_hi"]), int(c["key_lo"]))
        assert first[k] == int(c["first_start"])
        assert 0.0 <= c["F"] - fmin[k] <= 1e-9 * V
    assert np.all(copies["x"] <= 1.0) and np.all(copies["x"] >= 0.0)
    # a key reached by starts at different stationary points is rare
    assert np.mean(copies["flags"] & gc.GC_FLAG_COLLISION != 0) < 1e-3
    assert prog["sweeps_total"] == int(starts["sweeps32"].sum() + starts["sweeps64"].sum())
    assert prog["site_updates"] == prog["sweeps_total"] * V


@pytest.mark.parametrize("extent,n,omega,precision,sample", [
    ((4, 4, 4, 4), 100_000, 1.0, "fp64", 160),
    ((6, 6, 6, 6), 200_000, 1.7, "fp64", 300),
    ((10, 10, 10), 200_000, 1.7, "fp64", 300),
    ((6, 6, 6, 6), 200_000, 1.7, "mixed", 400),
    ((10, 10, 10), 200_000, 1.7, "mixed", 400),
])
def test_full_size_sampled_parity(ctx, extent, n, omega, precision, sample):
    phi = GI.orbit_angles(extent, 0, 0)
    p = gc.SolveParams(omega=omega, precision=precision)
    h, copies, starts, prog = run_gpu(ctx, extent, phi, n, p)
    assert prog["converged"] == n
    _check_table_properties(extent, copies, starts, prog)
    if precision == "fp64" and V_of(extent) <= 256:
        # the oracle runs every start of this workload in seconds: full parity,
        # lambda2 on a sample of copies and on every flagged copy
        note("oracle on all %d starts of %s" % (n, extent))
        flagged = {(int(c["key_hi"]), int(c["key_lo"])) for c in copies if c["flags"] & gc.GC_FLAG_COLLISION}
        pick = {(int(c["key_hi"]), int(c["key_lo"])) for c in copies[:: max(1, len(copies) // 24)]}
        o = O.enumerate_copies(extent, phi, np.arange(n), oracle_params(p), lambda_keys=flagged | pick)
        compare_starts(extent, starts, o["records"])
        compare_tables(extent, phi, copies, o, p, check_lambda=False)
        gk = {(int(c["key_hi"]), int(c["key_lo"])): c for c in copies}
        for k in flagged | pick:
            e = o["table"][k]
            assert abs(gk[k]["lambda2"] - e["lambda2"]) < LAMBDA_TOL
            assert (int(gk[k]["flags"]) & 15) == (e["flags"] & 15)
        # representatives fetched by key: copies whose lowest start is not
        # their representative (it halted next to a saddle), and a few others
        moved = [k for k, e in o["table"].items() if e["rep_start"] != e["first_start"]]
        for k in moved + sorted(pick)[:4]:
            e = o["table"][k]
            th = ctx.gc_fetch_state(h, k[0], k[1])
            _, gr, _ = O.solve(extent, phi, [e["rep_start"]], oracle_params(p), want_state=True)
            ref = O.theta_of(gr[0])
            d = np.angle(np.exp(1j * (th - (ref - ref[-1]))))
            assert np.max(np.abs(d)) < 1e-9 and th[-1] == 0.0
        with pytest.raises(gc.GcError) as err:
            ctx.gc_fetch_state(h, 1, 1)
        assert err.value.status == gc.GC_ENOTFOUND
        note("full parity: %d copies, %d flagged, %d with a moved representative" %
             (len(copies), len(flagged), len(moved)))
        ctx.gc_release(h)
        return
    ids = np.unique(np.concatenate([[0, n - 1], np.linspace(0, n - 1, sample).astype(np.int64)]))
    note("oracle on %d sampled starts of %s" % (ids.size, extent))
    o64, g64, _ = O.solve(extent, phi, ids, oracle_params(gc.SolveParams(omega=omega)), want_state=True)
    V = int(np.prod(extent))
    gs = starts[ids]
    same = (gs["key_hi"] == o64["key_hi"]) & (gs["key_lo"] == o64["key_lo"])
    if precision == "fp64":
        compare_starts(extent, gs, o64)
    else:
        # keys agree wherever the single-precision bulk reaches the double basin;
        # the FP32 rounding moves the basin of about 0.1 % of the starts on
        # these lattices, so more than 1 % of a 400-start sample is an error
        assert same.mean() >= 0.99
        assert np.max(np.abs(gs["F"][same] - o64["F"][same])) / V < F_TOL_PER_SITE
        # a start whose basin moved still converged to a genuine FP64 minimum
        land = BF.Landscape(extent, phi)
        for s in ids[~same][:4]:
            th = ctx.gc_fetch_start_state(h, int(s))
            grad = land.grad(th)
            assert np.mean(grad ** 2) < 2e-14
            r, _, _, w = O.observe(extent, phi, th)
            assert int(r["key_hi"]) == int(starts["key_hi"][s])
            lam0, lam2, _ = O.fp_spectrum(extent, w)
            assert lam2 > 0
        note("mixed: %d of %d sampled starts changed basin" % (int((~same).sum()), ids.size))
    # lambda2 of sampled copies against dense LAPACK on the oracle's own
    # double-precision solve of the copy's lowest start
    pick = copies[:: max(1, len(copies) // 12)][:12]
    ro, go, _ = O.solve(extent, phi, pick["first_start"], oracle_params(gc.SolveParams(omega=omega)),
                        want_state=True)
    for c, r, g in zip(pick, ro, go):
        if (int(r["key_hi"]), int(r["key_lo"])) != (int(c["key_hi"]), int(c["key_lo"])):
            continue      # mixed mode: this start's basin moved
        _, _, _, w = O.observe(extent, phi, O.theta_of(g))
        lam0, lam2, _ = O.fp_spectrum(extent, w)
        # FP64: same trajectory.  Mixed: a different path to the same minimum,
        # stopped at D < 1e-14, moves lambda2 to first order in the residual.
        tol = LAMBDA_TOL if precision == "fp64" else 4.0 * math.sqrt(V * 1e-14) / lam2
        assert abs(c["lambda2"] - lam2) < tol, (c["lambda2"], lam2)
        assert c["flags"] & gc.GC_FLAG_IN_REGION
    ctx.gc_release(h)


def test_batch_equals_single_launches(ctx):
    """Uneven orbits in one persistent graph launch give the same per-orbit
    results as launching each alone."""
    shapes = [((8, 8), 500), ((6, 6, 6), 300), ((4, 4, 4, 4), 200), ((3, 3), 100)]
    hs, singles = [], []
    for k, (ext, n) in enumerate(shapes):
        phi = GI.orbit_angles(ext, 0, k)
        h = ctx.gc_orbit_load(ext, phi, k)
        ctx.gc_launch(h, n, gc.SolveParams(omega=1.7))
        ctx.gc_wait(h)
        singles.append((ctx.gc_fetch(h), ctx.gc_fetch_starts(h, n)))
        hs.append(h)
    ctx.gc_launch_batch(hs, [n for _, n in shapes], gc.SolveParams(omega=1.7))
    for k, (ext, n) in enumerate(shapes):
        assert ctx.gc_wait(hs[k]) == gc.GC_OK
        c, s = ctx.gc_fetch(hs[k]), ctx.gc_fetch_starts(hs[k], n)
        assert np.array_equal(c[["key_hi", "key_lo", "hits", "first_start"]],
                              singles[k][0][["key_hi", "key_lo", "hits", "first_start"]])
        assert np.array_equal(s["key_hi"], singles[k][1]["key_hi"])
        assert np.array_equal(s["sweeps64"], singles[k][1]["sweeps64"])
        assert np.max(np.abs(c["F"] - singles[k][0]["F"])) < 1e-12
        ctx.gc_release(hs[k])


@pytest.mark.parametrize("omega", [1.7, 1.0])
def test_full_and_partial_slot_kernels_agree(ctx, omega):
    """6^4 (half volume 648) fills every slot of a lane but the last of the
    eleven-slot double-precision kernel: alone it runs the variant that tests
    only the last slot.  Batched with 6x6x6x4 (half volume 432: seven slots in
    the same kernel) the group runs the variant that tests every slot.  The
    6^4 starts come out bit for bit the same, final states included, and the
    partial orbit matches the oracle; over-relaxation and plain relaxation."""
    big, small = (6, 6, 6, 6), (6, 6, 6, 4)
    n_big, n_small = 300, 40
    p = gc.SolveParams(omega=omega)
    phi_b, phi_s = GI.orbit_angles(big, 2, 0), GI.orbit_angles(small, 2, 1)
    note("6^4 alone (%d starts, omega %s), then batched with 6x6x6x4" % (n_big, omega))
    hb = ctx.gc_orbit_load(big, phi_b, 0)
    ctx.gc_launch(hb, n_big, p)
    assert ctx.gc_wait(hb, 300_000) == gc.GC_OK
    alone = ctx.gc_fetch_starts(hb, n_big)
    alone_states = [ctx.gc_fetch_start_state(hb, s) for s in (0, 17, n_big - 1)]
    hs = ctx.gc_orbit_load(small, phi_s, 1)
    ctx.gc_launch_batch([hb, hs], [n_big, n_small], p)
    assert ctx.gc_wait(hb, 300_000) == gc.GC_OK and ctx.gc_wait(hs, 300_000) == gc.GC_OK
    both = ctx.gc_fetch_starts(hb, n_big)
    for f in ("status", "key_hi", "key_lo", "sweeps64", "F", "D"):
        assert np.array_equal(alone[f], both[f]), f
    for s, st in zip((0, 17, n_big - 1), alone_states):
        assert np.array_equal(ctx.gc_fetch_start_state(hb, s), st)
    o = O.enumerate_copies(small, phi_s, np.arange(n_small), oracle_params(p, 1))
    compare_starts(small, ctx.gc_fetch_starts(hs, n_small), o["records"])
    compare_tables(small, phi_s, ctx.gc_fetch(hs), o, p)
    ctx.gc_release(hb)
    ctx.gc_release(hs)


def test_saturation_curve_matches_oracle(ctx):
    """Distinct copies within the first 2^k starts (the paper's saturation
    curves), from the table's lowest start ids, against the oracle's table."""
    extent = (4, 4, 4)
    phi = GI.orbit_angles(extent, 3, 1)
    p = gc.SolveParams(omega=1.7, first_start=1000)
    h, copies, starts, _ = run_gpu(ctx, extent, phi, 3000, p, orbit_index=1)
    o = O.enumerate_copies(extent, phi, 1000 + np.arange(3000), oracle_params(p, 1))
    sizes = [1, 2, 4, 16, 64, 256, 1024, 2048, 3000]
    got = ctx.gc_saturation(h, sizes)
    got_in = ctx.gc_saturation(h, sizes, in_region_only=True)
    firsts = np.array([e["first_start"] - 1000 for e in o["table"].values()])
    firsts_in = np.array([e["first_start"] - 1000 for e in o["table"].values() if e["flags"] & O.FLAG_IN_REGION])
    for n, g, gi in zip(sizes, got, got_in):
        assert int(g) == int(np.sum(firsts < n)), n
        assert int(gi) == int(np.sum(firsts_in < n)), n
    assert int(got[-1]) == len(o["table"])
    assert np.all(np.diff(got.astype(np.int64)) >= 0)
    ctx.gc_release(h)


def test_paper_count_matches_oracle(ctx):
    """The paper's own count (distinct trunc(x * 1e8) over converged starts,
    Sec. III) within the first 2^k starts, counted on the device, against the
    oracle's records of the same starts; in the paper's mode (omega = 1,
    max |div| < 1e-12)."""
    extent = (4, 4)
    phi = GI.orbit_angles(extent, 5, 2)
    p = gc.SolveParams(omega=1.0, stop_norm="max_abs", eps64=1e-12)
    n = 4096
    h, copies, starts, prog = run_gpu(ctx, extent, phi, n, p, orbit_index=2)
    rec, _, _ = O.solve(extent, phi, np.arange(n), oracle_params(p, 2))
    sizes = [0, 1, 2, 4, 8, 16, 64, 256, 1024, 2048, 4096, 10000]
    got = ctx.gc_paper_saturation(h, sizes).astype(np.int64)
    conv_o = rec["status"] == O.CONVERGED
    conv_g = starts["status"] == gc.GC_START_CONVERGED
    # values differ between the two sides only where x * 1e8 lands within
    # rounding of an integer; each such start moves a count by at most one
    moved = int(np.sum(starts["paper_X"][conv_o] != rec["paper_X"][conv_o]))
    for m, g in zip(sizes, got):
        want = np.unique(rec["paper_X"][:m][conv_o[:m]]).size
        assert abs(int(g) - want) <= moved, (m, int(g), want)
        assert int(g) == np.unique(starts["paper_X"][:m][conv_g[:m]]).size, m
    assert int(got[-1]) == int(prog["paper_count"])
    assert np.all(np.diff(got) >= 0)
    with pytest.raises(gc.GcError):
        ctx.gc_paper_saturation(h, [4, 2])
    ctx.gc_release(h)


@pytest.mark.parametrize("extent,precision,n", [
    ((8, 8, 8), "fp64", 60),          # 256 slots per colour: two wavefronts per start
    ((10, 10, 10), "mixed", 40),      # 500: four
    ((6, 6, 6, 6), "mixed", 24),      # 648: six
    ((8, 8, 8, 8), "fp64", 3),        # 2048: sixteen
])
def test_parity_workgroup_per_start(monkeypatch, extent, precision, n):
    """The workgroup-per-start layout (forced for the context) against the
    oracle, start by start and copy by copy."""
    monkeypatch.setenv("GC_WPS", "1")
    phi = GI.orbit_angles(extent, 4, 2)
    p = gc.SolveParams(omega=1.7, precision=precision)
    with gc.Context(0) as c:
        h, copies, starts, _ = run_gpu(c, extent, phi, n, p, orbit_index=2)
        o = O.enumerate_copies(extent, phi, np.arange(n), oracle_params(p, 2))
        if precision == "fp64":
            compare_starts(extent, starts, o["records"])
            compare_tables(extent, phi, copies, o, p)
            check_start_filter(copies, starts, o)
        else:
            # mixed precision: keys agree start by start where the FP32 phase
            # reached the same basin; both sides' F agree on those
            conv = (o["records"]["status"] == O.CONVERGED) & (starts["status"] == gc.GC_START_CONVERGED)
            same = conv & (starts["key_hi"] == o["records"]["key_hi"]) & (starts["key_lo"] == o["records"]["key_lo"])
            assert same.sum() >= 0.97 * conv.sum()
            V = int(np.prod(extent))
            assert np.max(np.abs(starts["F"][same] - o["records"]["F"][same])) / V < F_TOL_PER_SITE
        c.gc_release(h)


@pytest.mark.parametrize("extent,mask,omega,n", [
    ((8,), 1, 1.0, 300),            # 1D ring: closed form below
    ((4, 6), 1, 1.7, 300),
    ((6, 6), 3, 1.0, 200),
    ((3, 3), 2, 1.7, 200),          # three colours
    ((4, 4, 4, 4), 5, 1.7, 300),
    ((6, 6, 6), 7, 1.0, 100),
])
def test_parity_antiperiodic(ctx, extent, mask, omega, n):
    """Antiperiodic gauge transformations in the directions of the mask
    (Sec. II): start by start and copy by copy against the oracle on the
    twisted orbit."""
    phi = GI.orbit_angles(extent, 2, 4)
    p = gc.SolveParams(omega=omega)
    note("antiperiodic extent=%s mask=%d" % (extent, mask))
    h = ctx.gc_orbit_load(extent, phi, 4, antiperiodic=mask)
    assert np.array_equal(ctx.gc_orbit_angles(h), phi)
    ctx.gc_launch(h, n, p)
    assert ctx.gc_wait(h, 600_000) == gc.GC_OK
    copies, starts = ctx.gc_fetch(h), ctx.gc_fetch_starts(h, n)
    o = O.enumerate_copies(extent, O.twisted(extent, phi, mask), np.arange(n), oracle_params(p, 4))
    compare_starts(extent, starts, o["records"])
    compare_tables(extent, phi, copies, o, p)
    check_start_filter(copies, starts, o)
    if len(extent) == 1:
        N = extent[0]
        Phi = float(np.sum(phi[0]))
        want = [N * (1 - math.cos((Phi + math.pi + 2 * math.pi * k) / N)) for k in range(-N - 1, N + 1)
                if abs(Phi + math.pi + 2 * math.pi * k) < N * math.pi / 2]
        for F in copies["F"]:
            assert min(abs(F - w) for w in want) < 1e-10
    ctx.gc_release(h)
    with pytest.raises(gc.GcError) as e:
        ctx.gc_orbit_load(extent, phi, 4, antiperiodic=1 << len(extent))
    assert e.value.status == gc.GC_EINVAL


@pytest.mark.parametrize("extent,batch,n,norm", [
    ((4, 4), 16, 200, "max_abs"),
    ((2, 2, 2, 2), 64, 300, "max_abs"),
    ((3, 3), 32, 100, "mean_sq"),
    ((4, 4, 4, 4), 1024, 3000, "max_abs"),
])
def test_parity_batch_synchronous_stop(ctx, extent, batch, n, norm):
    """The paper's batch-synchronous stop (Sec. III): every start of a batch
    runs as many sweeps as the batch's slowest; start by start against the
    oracle's two-pass definition."""
    phi = GI.orbit_angles(extent, 0, 6)
    eps = 1e-12 if norm == "max_abs" else 1e-14
    p = gc.SolveParams(omega=1.0, stop_norm=norm, eps64=eps, sync_batch=batch)
    note("sync extent=%s batch=%d n=%d" % (extent, batch, n))
    h = ctx.gc_orbit_load(extent, phi, 6)
    ctx.gc_launch(h, n, p)
    assert ctx.gc_wait(h, 600_000) == gc.GC_OK
    copies, starts, prog = ctx.gc_fetch(h), ctx.gc_fetch_starts(h, n), ctx.gc_poll(h)
    op = oracle_params(gc.SolveParams(omega=1.0, stop_norm=norm, eps64=eps), 6)
    pick = {(int(c["key_hi"]), int(c["key_lo"])) for c in copies[:: max(1, len(copies) // 16)]}
    o = O.enumerate_copies(extent, phi, np.arange(n), op, sync_batch=batch, lambda_keys=pick)
    compare_starts(extent, starts, o["records"])
    compare_tables(extent, phi, copies, o, p, check_lambda=False)
    for lo in range(0, n, batch):
        assert len(set(starts["sweeps64"][lo:lo + batch].tolist())) == 1
    assert prog["sweeps_total"] == int(starts["sweeps64"].sum())
    with pytest.raises(gc.GcError) as e:
        ctx.gc_launch(h, 10, gc.SolveParams(precision="mixed", sync_batch=8))
    assert e.value.status == gc.GC_EINVAL
    ctx.gc_release(h)
