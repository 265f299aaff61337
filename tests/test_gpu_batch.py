"""GPU: the uneven multi-orbit batch against the oracle.

The 32-orbit mix of lattices 8^2..16^2, 6^3, 8^3, 4^4 and 6^4 with 10^3..10^5
starts each goes through one gc_launch_batch (Sec. III replaces one fixed
grid of samples that waits for its slowest one; here every orbit's starts are
claimed dynamically inside one graph whose relax groups run concurrently).
Every orbit is compared with the oracle: the orbits of at most 256 sites start
by start with their whole copy table, the 512- and 1296-site orbits on
sampled starts; lambda2 of sampled copies against dense LAPACK.  A relaunch
of the same batch replays the captured graph and must reproduce the results
bit for bit."""
import sys

import numpy as np
import pytest

import gribov_inputs as GI
import paper_1403_0555_amd as gc
from oracle import oracle as O

pytestmark = pytest.mark.gpu

F_TOL_PER_SITE = 1e-10
LAMBDA_TOL = 1e-8


def note(msg):
    print("[gpu-batch] " + msg, flush=True)
    sys.stdout.flush()


def _key(c):
    return (int(c["key_hi"]), int(c["key_lo"]))


def _oparams(p, oi):
    return O.SolveParams(omega=p.omega, precision=p.precision, eps32=p.eps32, eps64=p.eps64,
                         start_seed=p.start_seed, orbit_index=oi)


def test_uneven_batch_matches_oracle():
    reqs = GI.uneven_batch(32)
    p = gc.SolveParams(omega=1.7)
    with gc.Context(0) as ctx:
        hs, phis = [], []
        for r in reqs:
            phi = GI.orbit_angles(r["extent"], r["seed"], r["orbit_index"])
            phis.append(phi)
            hs.append(ctx.gc_orbit_load(r["extent"], phi, r["orbit_index"]))
        note("batch of %d orbits, %d starts" % (len(reqs), sum(r["n_starts"] for r in reqs)))
        ctx.gc_launch_batch(hs, [r["n_starts"] for r in reqs], p)
        res = []
        for h, r in zip(hs, reqs):
            assert ctx.gc_wait(h, 600_000) == gc.GC_OK
            res.append((ctx.gc_fetch(h), ctx.gc_fetch_starts(h, r["n_starts"]), ctx.gc_poll(h)))
        lam_checked = 0
        for k, (r, phi, (copies, starts, prog)) in enumerate(zip(reqs, phis, res)):
            ext, n, oi = r["extent"], r["n_starts"], r["orbit_index"]
            V = int(np.prod(ext))
            keys = [_key(c) for c in copies]
            assert all(a < b for a, b in zip(keys, keys[1:]))
            assert prog["converged"] == n and int(copies["hits"].sum()) == n
            if V <= 256:
                # every start and the whole table; lambda2 on a sample of copies
                pick = set(keys[:: max(1, len(keys) // 6)])
                o = O.enumerate_copies(ext, phi, np.arange(n), _oparams(p, oi), lambda_keys=pick)
                rec = o["records"]
                assert np.array_equal(starts["status"], rec["status"])
                assert np.array_equal(starts["key_hi"], rec["key_hi"]) and np.array_equal(starts["key_lo"],
                                                                                           rec["key_lo"])
                dsw = np.abs(starts["sweeps64"].astype(np.int64) - rec["sweeps64"])
                assert dsw.max() <= 1 and np.mean(dsw == 0) > 0.99
                assert np.max(np.abs(starts["F"] - rec["F"])) / V < F_TOL_PER_SITE
                assert set(keys) == set(o["table"])
                for c in copies:
                    e = o["table"][_key(c)]
                    assert (int(c["hits"]), int(c["first_start"]), int(c["rep_start"])) == \
                        (e["hits"], e["first_start"], e["rep_start"])
                    assert abs(c["F"] - e["F"]) / V < F_TOL_PER_SITE
                    if "lambda2" in e:
                        assert abs(c["lambda2"] - e["lambda2"]) < LAMBDA_TOL
                        assert (int(c["flags"]) & 7) == (e["flags"] & 7)
                        lam_checked += 1
                note("orbit %d %s: %d starts, %d copies, oracle-identical" % (k, ext, n, len(copies)))
            else:
                ids = np.unique(np.concatenate([[0, n - 1], np.linspace(0, n - 1, 200).astype(np.int64)]))
                rec, g, _ = O.solve(ext, phi, ids, _oparams(p, oi), want_state=True)
                gs = starts[ids]
                assert np.array_equal(gs["status"], rec["status"])
                assert np.array_equal(gs["key_hi"], rec["key_hi"]) and np.array_equal(gs["key_lo"], rec["key_lo"])
                assert np.max(np.abs(gs["F"] - rec["F"])) / V < F_TOL_PER_SITE
                assert np.max(np.abs(gs["sweeps64"].astype(np.int64) - rec["sweeps64"])) <= 1
                # lambda2 of a few copies represented by sampled starts
                by_key = {_key(c): c for c in copies}
                done = 0
                for j, s in enumerate(ids):
                    c = by_key[(int(rec["key_hi"][j]), int(rec["key_lo"][j]))]
                    if int(c["rep_start"]) != int(s) or done >= 4:
                        continue
                    _, _, _, w = O.observe(ext, phi, O.theta_of(g[j]))
                    lam2 = O.fp_spectrum(ext, w)[1]
                    assert abs(c["lambda2"] - lam2) < LAMBDA_TOL
                    done += 1
                    lam_checked += 1
                note("orbit %d %s: %d sampled starts oracle-identical, lambda2 on %d" % (k, ext, ids.size, done))
        assert lam_checked >= 24
        # relaunch: the captured graph is replayed on the same block
        ctx.gc_launch_batch(hs, [r["n_starts"] for r in reqs], p)
        for h, r, (copies, starts, _) in zip(hs, reqs, res):
            assert ctx.gc_wait(h, 600_000) == gc.GC_OK
            c2, s2 = ctx.gc_fetch(h), ctx.gc_fetch_starts(h, r["n_starts"])
            for f in copies.dtype.names:
                assert np.array_equal(c2[f], copies[f], equal_nan=copies[f].dtype.kind == "f"), f
            for f in starts.dtype.names:
                assert np.array_equal(s2[f], starts[f], equal_nan=starts[f].dtype.kind == "f"), f
        for h in hs:
            ctx.gc_release(h)
