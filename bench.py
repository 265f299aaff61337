#!/usr/bin/env python3
"""Benchmark: random-start Gribov-copy enumeration of one orbit on one MI355X.

One step = the whole hot path for one orbit: random starts, checkerboard
relaxation (or over-relaxation) to the stopping threshold, functional and
integer key, copy-table insertion, Lanczos FP filter for each new copy, table
compaction and the sorted fetch to the host.  The default workload is the 4D
4^4 lattice with 1e5 starts, plain double-precision relaxation (omega = 1,
stop at mean |div|^2 < 1e-14).

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

# Algorithmic floating-point operations per site update, 16 d + 37: the
# staple S_i (2d complex multiply-adds, 16 d), its normalisation, the
# over-relaxation step and the divergence Im(conj(g_i) S_i) with its share of
# the stopping norm (37 together, counted once whatever omega is).
def flops_per_site_update(d: int) -> int:
    return 16 * d + 37


# HBM traffic of the relax kernel on the default workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by the same counters
# on a plain device copy of known size.  Valid only for the kernel sources
# they were taken on (SHA-256 of the relax sources below); otherwise null.
RELAX_SOURCES = ("gc_wave.hip", "gc_wave.h", "gc_common.h")
TRAFFIC = {"sources_sha256": "2edb455347f232feedb03e1b94b8a5187783a8448daf7b6bd1f8eda00ca165db",
           "bytes_per_launch": 429396470}


def relax_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in RELAX_SOURCES:
        with open(os.path.join(ROOT, "paper_1403_0555_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def relax_kernel_name(extent, tune) -> str:
    V = int(np.prod(extent))
    if all(e % 2 == 0 for e in extent):
        ns = (V // 2 + 63) // 64
        if ns <= 2 or not (tune and tune["relax_variant"] & 8):
            return "wave_kernel<%d, %d, 4, ...>" % (len(extent), min(ns, 32))
        wps = next(w for w in (2, 4, 6, 8, 16) if 2 * w >= ns)
        return "wps_kernel<%d, %d>" % (len(extent), wps)
    return "relax_wg_kernel<...>"


PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3


def cpu_baseline(w: GI.Workload, phi, n_sample: int):
    from oracle import oracle as O
    cores = os.cpu_count() or 1
    p = O.SolveParams(omega=w.omega, precision=w.precision, eps32=w.eps32, eps64=w.eps64,
                      start_seed=w.start_seed, orbit_index=w.orbit_index)
    t0 = time.perf_counter()
    res = O.enumerate_copies(w.extent, phi, np.arange(n_sample), p, threads=cores)
    dt = time.perf_counter() - t0
    rec = res["records"]
    inreg = 0
    for r in rec:
        if r["status"] == O.CONVERGED:
            e = res["table"][(int(r["key_hi"]), int(r["key_lo"]))]
            if e["flags"] & O.FLAG_IN_REGION:
                inreg += 1
    V = int(np.prod(w.extent))
    upd = int(rec["sweeps32"].sum() + rec["sweeps64"].sum()) * V
    return {"value": inreg / dt, "unit": "copies/s", "cores": cores, "kind": "oracle",
            "sample": "first %d starts of the same orbit and parameters (%.1f s)" % (n_sample, dt),
            "site_updates_per_s": upd / dt}


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
    """Uneven multi-orbit batch: every orbit's starts in one graph-captured launch."""
    reqs = GI.uneven_batch(32)
    params = gc.SolveParams(omega=1.7, precision=args.precision)
    ctx = gc.Context(0)
    hs = []
    for r in reqs:
        hs.append(ctx.gc_orbit_load(r["extent"], GI.orbit_angles(r["extent"], r["seed"], r["orbit_index"]),
                                    r["orbit_index"]))
    ns = [r["n_starts"] for r in reqs]
    V = [int(np.prod(r["extent"])) for r in reqs]

    def step():
        ctx.gc_launch_batch(hs, ns, params)
        for h in hs:
            if ctx.gc_wait(h, 600_000) != gc.GC_OK:
                raise RuntimeError("batch timed out")
        inreg = upd = dist = 0
        for h in hs:
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
        r = step()
        tot = [a + b for a, b in zip(tot, r)]
        print("batch step %d done" % k, file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    ctx.close()
    return {
        "metric": "converged Gribov copies/s", "value": tot[0] / wall, "unit": "copies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "uneven_batch_32_orbits", "orbits": len(reqs), "starts": int(sum(ns)),
                   "site_range": [min(V), max(V)], "omega": 1.7, "precision": args.precision},
        "site_updates_per_s": tot[1] / wall, "distinct_copies_per_s": tot[2] / wall,
    }


def run_serve(gc, args):
    """Serving stream: Poisson-arriving orbit requests, HBM-budget admission,
    continuous batching on the device; p50/p99 latency from submission to the
    orbit's final table."""
    import threading
    probe = GI.poisson_requests(args.requests, 1.0, seed=1)
    # capacity estimate: starts/s measured on a short warmup request mix
    params = gc.SolveParams(omega=1.7, precision=args.precision)
    ctx = gc.Context(0, hbm_budget_bytes=int(args.budget_gb * (1 << 30)))
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
    lat, results = [], []
    lock = threading.Lock()
    handles = []
    t_start = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t_start
        if r["t_arrive"] > now:
            time.sleep(r["t_arrive"] - now)
        h = ctx.gc_orbit_load(r["extent"], GI.orbit_angles(r["extent"], r["seed"], r["orbit_index"]), r["orbit_index"])
        ctx.gc_launch(h, r["n_starts"], params)
        handles.append(h)
        # release finished orbits as we go (frees their HBM for admission)
        done = []
        for hh in handles:
            if ctx.gc_poll(hh)["state"] == gc.GC_ORBIT_DONE:
                done.append(hh)
        for hh in done:
            p = ctx.gc_poll(hh)
            c = ctx.gc_fetch(hh)
            results.append((p, c))
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
    return {
        "metric": "converged Gribov copies/s", "value": inreg / wall, "unit": "copies/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "serving_poisson", "requests": len(reqs), "offered_load": args.load,
                   "rate_per_s": rate, "budget_gb": args.budget_gb, "omega": 1.7, "precision": args.precision},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "site_updates_per_s": upd / wall,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="u1_4d_4x4x4x4_relax",
                    choices=sorted(GI.WORKLOADS) + ["batch", "serve", "copy"])
    ap.add_argument("--copy-mib", type=int, default=2048, help="copy mode: bytes per copy, MiB")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"], help="batch/serve modes")
    ap.add_argument("--requests", type=int, default=300, help="serve mode")
    ap.add_argument("--load", type=float, default=0.8, help="serve mode: offered load / capacity")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve mode")
    ap.add_argument("--starts", type=int, default=0, help="override the workload's start count")
    ap.add_argument("--cpu-sample", type=int, default=5000, help="oracle sample: first N starts (10-30 s on 16 threads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the kernel-variant autotuner")
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
    phi = GI.orbit_angles(w.extent, w.seed, w.orbit_index)
    params = gc.SolveParams(omega=w.omega, precision=w.precision, eps32=w.eps32, eps64=w.eps64,
                            start_seed=w.start_seed)

    ctx = gc.Context(0)
    inflight = max(1, args.inflight)
    # every handle holds the same orbit, so every step computes the same result
    hs = [ctx.gc_orbit_load(w.extent, phi, w.orbit_index) for _ in range(inflight)]
    tune = None
    if not args.no_tune:
        # kernel variants for this shape, chosen before timing on launches
        # of the same size as the timed ones
        tune = ctx.gc_autotune(hs[0], n, params)
        print("autotune: %s" % tune, file=sys.stderr, flush=True)

    t_launch = [0.0] * inflight

    def launch(i):
        t_launch[i] = time.perf_counter()
        ctx.gc_launch(hs[i], n, params)

    def finish(i):
        if ctx.gc_wait(hs[i], 600_000) != gc.GC_OK:
            raise RuntimeError("launch timed out")
        copies = ctx.gc_fetch(hs[i])
        return copies, ctx.gc_poll(hs[i]), ctx.gc_kernel_time_ms(hs[i])

    for k in range(args.warmup):
        launch(0)
        finish(0)
        print("warmup step %d done" % k, file=sys.stderr, flush=True)

    lat, kms, conv_inreg, upd, distinct = [], [], 0, 0, 0
    t0 = time.perf_counter()
    for i in range(min(inflight, args.steps)):
        launch(i)
    for k in range(args.steps):
        i = k % inflight
        copies, prog, solve_ms = finish(i)
        lat.append((time.perf_counter() - t_launch[i]) * 1e3)
        if k + inflight < args.steps:
            launch(i)
        kms.append(solve_ms)
        inreg = copies["flags"] & gc.GC_FLAG_IN_REGION != 0
        conv_inreg += int(copies["hits"][inreg].sum())
        upd += int(prog["site_updates"])
        distinct += len(copies)
        print("step %d: %.1f ms, solve kernel %.1f ms, %d copies" % (k, lat[-1], solve_ms, len(copies)),
              file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    for h in hs:
        ctx.gc_release(h)
    ctx.close()

    fl = flops_per_site_update(d)
    mean_kernel_s = float(np.mean(kms)) / 1e3
    if inflight > 1:
        # concurrent launches share the chip, so one launch's kernel time no
        # longer measures the kernel: charge the wall clock per step instead
        mean_kernel_s = wall / args.steps
    upd_per_launch = upd / args.steps
    achieved_tflops = fl * upd_per_launch / mean_kernel_s / 1e12
    peak = PEAK_FP64_TFLOPS if w.precision == "fp64" else PEAK_FP32_TFLOPS
    traffic = None
    if (args.workload == "u1_4d_4x4x4x4_relax" and not args.starts and inflight == 1 and TRAFFIC["sources_sha256"]
            and TRAFFIC["sources_sha256"] == relax_sources_sha256()):
        traffic = TRAFFIC["bytes_per_launch"]
    out = {
        "metric": "converged Gribov copies/s",
        "value": conv_inreg / wall,
        "unit": "copies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "extent": list(w.extent), "n_starts": n, "omega": w.omega,
                   "precision": w.precision, "eps64": w.eps64, "eps32": w.eps32,
                   "orbit_seed": w.seed, "start_seed": w.start_seed, "inflight": inflight},
        "site_updates_per_s": upd / wall,
        "distinct_copies_per_s": distinct / wall,
        "autotune": tune,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "solve_kernel_ms": float(np.mean(kms)),
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved_tflops / peak, "traffic": traffic,
                     "kernel": relax_kernel_name(w.extent, tune), "kernel_ms": float(np.mean(kms)),
                     "flops_per_site_update": fl, "site_updates_per_launch": upd_per_launch,
                     "time_basis": "kernel" if inflight == 1 else "wall per step"},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, phi, min(args.cpu_sample, n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
