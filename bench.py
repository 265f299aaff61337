#!/usr/bin/env python3
"""Benchmark: random-start Gribov-copy enumeration of one orbit on one MI355X.

One step = the whole hot path for one orbit: random starts, checkerboard
relaxation (or over-relaxation) to the stopping threshold, functional and
integer key, copy-table insertion, Lanczos FP filter for each new copy, table
compaction and the sorted fetch to the host.  The default workload is the 4D
6^4 lattice with 10^6 starts in double precision throughout (the paper's
precision), over-relaxation omega = 1.7, stop at mean |div|^2 < 1e-14.  The
same orbit and starts are then run with single-precision bulk sweeps and a
double-precision polish, and compared start by start with the double run
(the single-precision error of that result), and the 3D 10^3 lattice is run
both ways as well.

Prints one JSON line.  ``value`` is converged copies/s: starts that converged
to a copy inside the first Gribov region, per second of wall time.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gribov_inputs as GI  # noqa: E402

DEFAULT_WORKLOAD = "u1_4d_6x6x6x6_fp64"
TWINS = {"u1_4d_6x6x6x6_fp64": "u1_4d_6x6x6x6_mixed", "u1_4d_6x6x6x6_mixed": "u1_4d_6x6x6x6_fp64",
         "u1_3d_10x10x10_fp64": "u1_3d_10x10x10_mixed", "u1_3d_10x10x10_mixed": "u1_3d_10x10x10_fp64"}

PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3


def relax_flops_per_site_update(d: int, omega: float) -> int:
    """Algorithmic floating-point operations of one site update: the staple
    S_i (2d complex multiply-adds, 16 d), its normalisation (8) and the
    divergence Im(conj(g_i) S_i) with its share of the stopping norm (5);
    over-relaxation (omega != 1) adds the interpolation (1 - omega) g +
    omega S/|S| (4) and its normalisation (7)."""
    return 16 * d + 13 + (0 if omega == 1.0 else 11)


def lanczos_flops_per_site(d: int) -> int:
    """Algorithmic floating-point operations per site and Lanczos iteration
    of the FP filter: the matrix-vector product with M = B^T diag(w) B, two
    link terms w (q_i - q_j) per direction (6 d), the three dot products of
    the iteration (5), the three-term residual (5), its norm (2) and the
    scaling of the next basis vector (1)."""
    return 6 * d + 13


# HBM traffic of the dominant kernel per launch, from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE) over the default workload, each scaled by
# the same counter on a plain device copy of known size.  Valid only for the
# kernel sources they were taken on (SHA-256 below); otherwise null.
KERNEL_SOURCES = {
    "relax": ("gc_wave_kern.h", "gc_wave.h", "gc_wave4.hip", "gc_common.h", "gc_internal.h"),
    "lanczos_kernel": ("gc_lanczos_kern.h", "gc_filter.h", "gc_lanczos4.hip", "gc_common.h", "gc_internal.h"),
}
TRAFFIC = {
    # wave_rr_kernel<4, 11, 8> (exact-slot variant), 10^6 starts of the 6^4
    # FP64 workload (one dispatch): FETCH_SIZE 665782.7 KiB x 2.0000 (a 2 GiB
    # copy reads 1048587.5 KiB) and WRITE_SIZE 20538190.2 KiB x 1.0 (the copy
    # writes 2097152.0 KiB); the sources have since changed in other kernels
    # only (this kernel's assembly is unchanged)
    "sources_sha256": "9397f846b062f06c8b80ecc8552275f05cda6f2d53713d940c0e7f84710d6c44",
    "kernel": "relax",
    "bytes_per_launch": 1363522944 + 21031106752,
}


def kernel_sources_sha256(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, ()):
        with open(os.path.join(ROOT, "paper_1403_0555_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_leg(O, w, phi, ids, threads):
    p = O.SolveParams(omega=w.omega, precision=w.precision, eps32=w.eps32, eps64=w.eps64,
                      start_seed=w.start_seed, orbit_index=w.orbit_index)
    t0 = time.perf_counter()
    res = O.enumerate_copies(w.extent, phi, ids, p, threads=threads)
    dt = time.perf_counter() - t0
    rec = res["records"]
    inreg = sum(1 for r in rec if r["status"] == O.CONVERGED and
                res["table"][(int(r["key_hi"]), int(r["key_lo"]))]["flags"] & O.FLAG_IN_REGION)
    upd = int(rec["sweeps32"].sum() + rec["sweeps64"].sum()) * int(np.prod(w.extent))
    return inreg / dt, upd / dt, dt


def cpu_baseline(w, phi, n_sample: int, n_single: int):
    """The oracle as it stands (C relaxation with OpenMP over starts, dense
    LAPACK eigenvalues for the FP filter) on the first starts of the same
    workload, on every host core, and on one core."""
    from oracle import oracle as O
    from threadpoolctl import threadpool_limits
    cores = host_cores()
    v, su, dt = _oracle_leg(O, w, phi, np.arange(n_sample), cores)
    with threadpool_limits(1):
        v1, su1, dt1 = _oracle_leg(O, w, phi, np.arange(n_single), 1)
    return {"value": v, "unit": "copies/s", "cores": cores, "kind": "oracle",
            "sample": "first %d starts of the same orbit and parameters, %.1f s on %d threads (%s); "
                      "relaxation in C, lambda2 of every copy by dense LAPACK" % (n_sample, dt, cores, cpu_model()),
            "site_updates_per_s": su, "cpu_model": cpu_model(),
            "single_core": {"value": v1, "site_updates_per_s": su1,
                            "sample": "first %d starts, %.1f s" % (n_single, dt1)}}


def run_workload(gc, ctx, w, n, steps, warmup, tune_n, inflight=1, keep_starts=False, label=""):
    """Timed steps of one workload; returns the measurements (and the last
    step's per-start records and copies when keep_starts)."""
    phi = GI.orbit_angles(w.extent, w.seed, w.orbit_index)
    params = gc.SolveParams(omega=w.omega, precision=w.precision, eps32=w.eps32, eps64=w.eps64,
                            start_seed=w.start_seed)
    hs = [ctx.gc_orbit_load(w.extent, phi, w.orbit_index) for _ in range(inflight)]
    # one host buffer per launch in flight, reused by every fetch (at most
    # one copy per start); the warmup touches its pages
    bufs = [np.zeros(n, dtype=gc.COPY_DTYPE) for _ in range(inflight)]
    tune = None
    if tune_n:
        tune = ctx.gc_autotune(hs[0], min(n, tune_n), params)
        print("%sautotune: %s" % (label, tune), file=sys.stderr, flush=True)
    t_launch = [0.0] * inflight

    def launch(i):
        t_launch[i] = time.perf_counter()
        ctx.gc_launch(hs[i], n, params)

    def finish(i):
        if ctx.gc_wait(hs[i], 600_000) != gc.GC_OK:
            raise RuntimeError("launch timed out")
        return ctx.gc_fetch(hs[i], out=bufs[i]), ctx.gc_poll(hs[i])

    for k in range(warmup):
        launch(0)
        finish(0)
        print("%swarmup step %d done" % (label, k), file=sys.stderr, flush=True)
    lat, kms, pms, fms, conv_inreg, upd, distinct, lits = [], [], [], [], 0, 0, 0, 0
    last = None
    t0 = time.perf_counter()
    for i in range(min(inflight, steps)):
        launch(i)
    for k in range(steps):
        i = k % inflight
        copies, prog = finish(i)
        lat.append((time.perf_counter() - t_launch[i]) * 1e3)
        if keep_starts and k == steps - 1:
            last = (copies, i)   # a view of bufs[i]: nothing is fetched into it after the last step
        if k + inflight < steps:
            launch(i)
        kms.append(prog["device_ms"])
        pms.append(prog["post_ms"])
        fms.append(prog["filter_ms"])
        conv_inreg += int(prog["in_region_hits"])
        upd += int(prog["site_updates"])
        distinct += len(copies)
        lits += int(prog["lanczos_iters"])
        print("%sstep %d: %.1f ms, relax %.1f ms, key pass %.1f ms, filter %.1f ms, %d copies" %
              (label, k, lat[-1], kms[-1], pms[-1], fms[-1], len(copies)), file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    if last is not None:
        # the per-start records of the last step, for the precision
        # comparison: read after the clock stops (not part of the workload)
        last = (last[0], ctx.gc_fetch_starts(hs[last[1]], n))
    for h in hs:
        ctx.gc_release(h)
    return {"phi": phi, "tune": tune, "wall": wall, "steps": steps, "lat": lat, "relax_ms": kms, "post_ms": pms,
            "filter_ms": fms,
            "conv_inreg": conv_inreg, "site_updates": upd, "distinct": distinct, "lanczos_iters": lits,
            "last": last, "inflight": inflight}


def su2_reduction(gc, ctx, extent):
    """The maximal Abelian reduction of a Haar-random SU(2) configuration on
    the lattice of the workload (once per configuration, before enumeration):
    wall time of gc_orbit_load_su2 after a first call, sweeps and R/(dV)."""
    links = GI.su2_links(extent, 0, 0)
    ctx.gc_release(ctx.gc_orbit_load_su2(extent, links)[0])
    t0 = time.perf_counter()
    h, info = ctx.gc_orbit_load_su2(extent, links)
    ms = (time.perf_counter() - t0) * 1e3
    ctx.gc_release(h)
    return {"load_ms": ms, "sweeps": info["sweeps"], "R": info["R"], "converged": info["converged"]}


def compare_precisions(w, r64, rmx):
    """Single-precision error of the mixed result, start by start against the
    double-precision run of the same orbit and starts."""
    (c64, s64), (cmx, smx) = r64["last"], rmx["last"]
    V = int(np.prod(w.extent))
    conv = (s64["status"] == 1) & (smx["status"] == 1)
    same = conv & (s64["key_hi"] == smx["key_hi"]) & (s64["key_lo"] == smx["key_lo"])
    k64 = set(zip(c64["key_hi"].tolist(), c64["key_lo"].tolist()))
    kmx = set(zip(cmx["key_hi"].tolist(), cmx["key_lo"].tolist()))
    return {"starts": int(len(s64)), "flips": int(conv.sum() - same.sum()),
            "flip_fraction": float(1.0 - same.sum() / max(1, conv.sum())),
            "max_abs_dF_per_site_same_basin": float(np.max(np.abs(s64["F"][same] - smx["F"][same])) / V)
            if same.any() else None,
            "copies_fp64_only": len(k64 - kmx), "copies_mixed_only": len(kmx - k64)}


def summary(w, r):
    steps = r["steps"]
    return {"copies_per_s": r["conv_inreg"] / r["wall"], "ms_per_step": r["wall"] / steps * 1e3,
            "site_updates_per_s": r["site_updates"] / r["wall"], "distinct_copies_per_s": r["distinct"] / r["wall"],
            "relax_ms": float(np.mean(r["relax_ms"])), "key_pass_ms": float(np.mean(r["post_ms"])),
            "filter_ms": float(np.mean(r["filter_ms"])), "steps": steps,
            "autotune": r["tune"]}


def rooflines(w, r):
    """ALU rooflines of the relax kernel and the FP filter kernel:
    algorithmic flops per launch over the kernel's mean duration (HIP events
    on its stream)."""
    d = len(w.extent)
    V = int(np.prod(w.extent))
    steps = r["steps"]
    relax_s = float(np.mean(r["relax_ms"])) / 1e3
    post_s = float(np.mean(r["filter_ms"])) / 1e3
    su = r["site_updates"] / steps
    rf = relax_flops_per_site_update(d, w.omega)
    peak_relax = PEAK_FP64_TFLOPS if w.precision == "fp64" else PEAK_FP32_TFLOPS
    relax = {"bound": "alu", "achieved": rf * su / relax_s / 1e12, "peak": peak_relax, "unit": "TFLOP/s",
             "kernel": "relax", "kernel_ms": relax_s * 1e3, "flops_per_site_update": rf,
             "site_updates_per_launch": su}
    relax["frac"] = relax["achieved"] / peak_relax
    lits = r["lanczos_iters"] / steps
    lf = lanczos_flops_per_site(d)
    post = {"bound": "alu", "achieved": lf * V * lits / post_s / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "kernel": "lanczos_kernel", "kernel_ms": post_s * 1e3, "flops_per_site_iteration": lf,
            "lanczos_iterations_per_launch": lits, "sites": V}
    post["frac"] = post["achieved"] / PEAK_FP64_TFLOPS
    return relax, post


def run_copy(args):
    """Plain device-to-device copy of a known size: the calibration run for
    the HBM byte counters (FETCH_SIZE / WRITE_SIZE per dispatch)."""
    import torch
    n = (args.copy_mib << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    nbytes = 4 * n
    return {"metric": "device copy bandwidth", "value": 2 * nbytes / dt / 1e9, "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "copy", "bytes_read": nbytes, "bytes_written": nbytes}}


def run_batch(gc, args):
    """The uneven 32-orbit batch (8^2..16^2, 6^3, 8^3, 4^4, 6^4; 10^3..10^5
    starts each) in one graph-captured launch per step, mixed precision and
    double precision on the same orbits; each distinct shape autotuned first."""
    reqs = GI.uneven_batch(32)
    ctx = gc.Context(0, tune_cache=args.tune_cache)
    hs = [ctx.gc_orbit_load(r["extent"], GI.orbit_angles(r["extent"], r["seed"], r["orbit_index"]), r["orbit_index"])
          for r in reqs]
    ns = [r["n_starts"] for r in reqs]
    V = [int(np.prod(r["extent"])) for r in reqs]
    out = {}
    for prec in ("mixed", "fp64"):
        params = gc.SolveParams(omega=1.7, precision=prec)
        if not args.no_tune:
            seen = set()
            for h, r in zip(hs, reqs):
                if r["extent"] not in seen:
                    seen.add(r["extent"])
                    ctx.gc_autotune(h, min(r["n_starts"], 20000), params)

        def step():
            ctx.gc_launch_batch(hs, ns, params)
            inreg = upd = dist = 0
            for h in hs:
                if ctx.gc_wait(h, 600_000) != gc.GC_OK:
                    raise RuntimeError("batch timed out")
                c = ctx.gc_fetch(h)
                inreg += int(c["hits"][(c["flags"] & gc.GC_FLAG_IN_REGION) != 0].sum())
                dist += len(c)
                upd += int(ctx.gc_poll(h)["site_updates"])
            return inreg, upd, dist

        for _ in range(args.warmup):
            step()
        t0 = time.perf_counter()
        tot = [0, 0, 0]
        for k in range(args.steps):
            tot = [a + b for a, b in zip(tot, step())]
            print("batch %s step %d done" % (prec, k), file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        out[prec] = {"copies_per_s": tot[0] / wall, "ms_per_step": wall / args.steps * 1e3,
                     "site_updates_per_s": tot[1] / wall, "distinct_copies_per_s": tot[2] / wall}
    ctx.close()
    m = out["mixed"]
    return {
        "metric": "converged Gribov copies/s", "value": m["copies_per_s"], "unit": "copies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "uneven_batch_32_orbits", "orbits": len(reqs), "starts": int(sum(ns)),
                   "site_range": [min(V), max(V)], "omega": 1.7, "precision": "mixed"},
        "site_updates_per_s": m["site_updates_per_s"], "distinct_copies_per_s": m["distinct_copies_per_s"],
        "fp64": out["fp64"], "mixed_over_fp64": m["copies_per_s"] / out["fp64"]["copies_per_s"],
    }


def run_serve(gc, args):
    """Serving stream: Poisson-arriving orbit requests drawn from the batch
    shapes (10^3..10^5 starts) and the 4D 8^4 lattice with 10^4 starts, HBM
    budget admission, continuous batching on the device; p50/p99 latency from
    submission to the orbit's final table, finished orbits fetched and
    released while others run."""
    probe = GI.poisson_requests(args.requests, 1.0, seed=1)
    params = gc.SolveParams(omega=1.7, precision=args.precision)
    ctx = gc.Context(0, hbm_budget_bytes=int(args.budget_gb * (1 << 30)), tune_cache=args.tune_cache)
    # capacity estimate: site-starts per second over a short sequential mix
    work = sum(r["n_starts"] * int(np.prod(r["extent"])) for r in probe)
    t0 = time.perf_counter()
    for r in probe[:8]:
        h = ctx.gc_orbit_load(r["extent"], GI.orbit_angles(r["extent"], r["seed"], r["orbit_index"]), r["orbit_index"])
        ctx.gc_launch(h, r["n_starts"], params)
        ctx.gc_wait(h)
        ctx.gc_release(h)
    cap_sites = sum(r["n_starts"] * int(np.prod(r["extent"])) for r in probe[:8]) / (time.perf_counter() - t0)
    rate = args.load * cap_sites / (work / len(probe))
    reqs = GI.poisson_requests(args.requests, rate, seed=1)
    results, handles, launch_ms = [], [], []
    t_start = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t_start
        if r["t_arrive"] > now:
            time.sleep(r["t_arrive"] - now)
        h = ctx.gc_orbit_load(r["extent"], GI.orbit_angles(r["extent"], r["seed"], r["orbit_index"]), r["orbit_index"])
        tl = time.perf_counter()
        ctx.gc_launch(h, r["n_starts"], params)
        launch_ms.append((time.perf_counter() - tl) * 1e3)
        handles.append(h)
        done = [hh for hh in handles if ctx.gc_poll(hh)["state"] == gc.GC_ORBIT_DONE]
        for hh in done:
            results.append((ctx.gc_poll(hh), ctx.gc_fetch(hh)))
            ctx.gc_release(hh)
            handles.remove(hh)
    for hh in handles:
        ctx.gc_wait(hh)
        results.append((ctx.gc_poll(hh), ctx.gc_fetch(hh)))
        ctx.gc_release(hh)
    wall = time.perf_counter() - t_start
    ctx.close()
    lat = [p["submit_to_done_ms"] for p, _ in results]
    inreg = sum(int(c["hits"][(c["flags"] & gc.GC_FLAG_IN_REGION) != 0].sum()) for _, c in results)
    upd = sum(int(p["site_updates"]) for p, _ in results)
    n8 = sum(1 for r in reqs if len(r["extent"]) == 4 and r["extent"][0] == 8)
    return {
        "metric": "converged Gribov copies/s", "value": inreg / wall, "unit": "copies/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "serving_poisson", "requests": len(reqs), "requests_8x8x8x8": n8,
                   "offered_load": args.load, "rate_per_s": rate, "budget_gb": args.budget_gb, "omega": 1.7,
                   "precision": args.precision},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "gc_launch_ms": {"p50": float(np.percentile(launch_ms, 50)), "max": float(np.max(launch_ms))},
        "site_updates_per_s": upd / wall,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
                    choices=sorted(GI.WORKLOADS) + ["batch", "serve", "copy"])
    ap.add_argument("--copy-mib", type=int, default=2048, help="copy mode: bytes per copy, MiB")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"], help="serve mode")
    ap.add_argument("--requests", type=int, default=300, help="serve mode")
    ap.add_argument("--load", type=float, default=0.8, help="serve mode: offered load / capacity")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve mode")
    ap.add_argument("--starts", type=int, default=0, help="override the workload's start count")
    ap.add_argument("--tune-starts", type=int, default=100_000, help="autotuner launch size")
    ap.add_argument("--extra-steps", type=int, default=2,
                    help="timed steps of the comparison runs (the other precision, the 10^3 lattice)")
    ap.add_argument("--no-extra", action="store_true", help="skip the comparison runs")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample: first N starts (0: by lattice size)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the kernel-variant autotuner")
    ap.add_argument("--tune-cache", default=None, help="file the autotuner's choices persist in")
    ap.add_argument("--inflight", type=int, default=1,
                    help="launches of the workload kept in flight (each a full step on its own orbit handle); "
                         "above 1, one launch's slowest starts overlap the next launch's bulk")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: each start is independent and the path needs no "
              "collective; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "copy":
        print(json.dumps(run_copy(args)), flush=True)
        return

    import paper_1403_0555_amd as gc

    if args.workload in ("batch", "serve"):
        out = run_batch(gc, args) if args.workload == "batch" else run_serve(gc, args)
        print(json.dumps(out), flush=True)
        return

    w = GI.WORKLOADS[args.workload]
    n = args.starts or w.n_starts
    d = len(w.extent)
    V = int(np.prod(w.extent))
    tune_n = 0 if args.no_tune else args.tune_starts
    ctx = gc.Context(0, tune_cache=args.tune_cache)
    extra = {}
    twin = TWINS.get(args.workload) if not args.no_extra else None
    r = run_workload(gc, ctx, w, n, args.steps, args.warmup, tune_n, inflight=max(1, args.inflight),
                     keep_starts=twin is not None and args.inflight == 1)
    if twin:
        wt = GI.WORKLOADS[twin]
        rt = run_workload(gc, ctx, wt, n, args.extra_steps, 1, tune_n, keep_starts=True, label="[%s] " % twin)
        r64, rmx = (r, rt) if w.precision == "fp64" else (rt, r)
        extra[wt.precision] = summary(wt, rt)
        extra["fp32_error"] = compare_precisions(w, r64, rmx)
        extra["mixed_over_fp64"] = (rmx["conv_inreg"] / rmx["wall"]) / (r64["conv_inreg"] / r64["wall"])
        rt["last"] = None
        if d == 4:
            # the other lattice of the same configuration, both precisions
            w3, w3m = GI.WORKLOADS["u1_3d_10x10x10_fp64"], GI.WORKLOADS["u1_3d_10x10x10_mixed"]
            a = run_workload(gc, ctx, w3, n, args.extra_steps, 1, tune_n, keep_starts=True, label="[10^3 fp64] ")
            b = run_workload(gc, ctx, w3m, n, args.extra_steps, 1, tune_n, keep_starts=True, label="[10^3 mixed] ")
            extra["lattice_10x10x10"] = {"fp64": summary(w3, a), "mixed": summary(w3m, b),
                                         "fp32_error": compare_precisions(w3, a, b),
                                         "mixed_over_fp64": (b["conv_inreg"] / b["wall"]) /
                                                            (a["conv_inreg"] / a["wall"])}
            extra["su2_maximal_abelian_6x6x6x6"] = su2_reduction(gc, ctx, w.extent)
    ctx.close()

    relax, post = rooflines(w, r)
    inflight = r["inflight"]
    if inflight > 1:
        # concurrent launches share the chip: charge the wall clock per step
        for rf in (relax, post):
            rf["achieved"] *= rf["kernel_ms"] / (r["wall"] / r["steps"] * 1e3)
            rf["frac"] = rf["achieved"] / rf["peak"]
            rf["time_basis"] = "wall per step"
    dominant, other = (post, relax) if post["kernel_ms"] >= relax["kernel_ms"] else (relax, post)
    traffic = None
    if (TRAFFIC["bytes_per_launch"] and args.workload == DEFAULT_WORKLOAD and not args.starts and inflight == 1
            and TRAFFIC["kernel"] == dominant["kernel"]
            and TRAFFIC["sources_sha256"] == kernel_sources_sha256(dominant["kernel"])):
        traffic = TRAFFIC["bytes_per_launch"]
    dominant["traffic"] = traffic
    wall, steps = r["wall"], r["steps"]
    out = {
        "metric": "converged Gribov copies/s",
        "value": r["conv_inreg"] / wall,
        "unit": "copies/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "extent": list(w.extent), "n_starts": n, "omega": w.omega,
                   "precision": w.precision, "eps64": w.eps64, "eps32": w.eps32,
                   "orbit_seed": w.seed, "start_seed": w.start_seed, "inflight": inflight},
        "site_updates_per_s": r["site_updates"] / wall,
        "distinct_copies_per_s": r["distinct"] / wall,
        "autotune": r["tune"],
        "latency_ms": {"p50": float(np.percentile(r["lat"], 50)), "p99": float(np.percentile(r["lat"], 99))},
        "relax_kernel_ms": float(np.mean(r["relax_ms"])),
        "key_pass_ms": float(np.mean(r["post_ms"])),
        "filter_kernel_ms": float(np.mean(r["filter_ms"])),
        "roofline": dominant,
        "roofline_other_kernel": other,
    }
    out.update(extra)
    if not args.no_cpu:
        # about 10-20 s of oracle work on the machine's host threads, a few
        # seconds on one core
        n_sample = args.cpu_sample or (5000 if V <= 256 else 144)
        out["cpu_baseline"] = cpu_baseline(w, r["phi"], min(n_sample, n), 16 if V > 256 else 200)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
