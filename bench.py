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

# Algorithmic floating-point operations per site update (a multiply or an add
# counts one, a reciprocal square root one): the update S_i (16 d), its
# normalisation (6), the over-relaxation step (22, omega != 1), and the
# stopping test on the post-sweep state evaluated every sweep (16 d + 5).
def flops_per_site_update(d: int, omega: float) -> int:
    return 32 * d + 11 + (22 if omega != 1.0 else 0)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="u1_4d_4x4x4x4_relax", choices=sorted(GI.WORKLOADS))
    ap.add_argument("--starts", type=int, default=0, help="override the workload's start count")
    ap.add_argument("--cpu-sample", type=int, default=2000)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: each start is independent and the path needs no "
              "collective; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import paper_1403_0555_amd as gc

    w = GI.WORKLOADS[args.workload]
    n = args.starts or w.n_starts
    d = len(w.extent)
    V = int(np.prod(w.extent))
    phi = GI.orbit_angles(w.extent, w.seed, w.orbit_index)
    params = gc.SolveParams(omega=w.omega, precision=w.precision, eps32=w.eps32, eps64=w.eps64,
                            start_seed=w.start_seed)

    ctx = gc.Context(0)
    h = ctx.gc_orbit_load(w.extent, phi, w.orbit_index)

    def step():
        ctx.gc_launch(h, n, params)
        if ctx.gc_wait(h, 600_000) != gc.GC_OK:
            raise RuntimeError("launch timed out")
        copies = ctx.gc_fetch(h)
        return copies, ctx.gc_poll(h), ctx.gc_kernel_time_ms(h)

    for k in range(args.warmup):
        step()
        print("warmup step %d done" % k, file=sys.stderr, flush=True)

    lat, kms, conv_inreg, upd, distinct = [], [], 0, 0, 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        copies, prog, solve_ms = step()
        lat.append((time.perf_counter() - ts) * 1e3)
        kms.append(solve_ms)
        inreg = copies["flags"] & gc.GC_FLAG_IN_REGION != 0
        conv_inreg += int(copies["hits"][inreg].sum())
        upd += int(prog["site_updates"])
        distinct += len(copies)
        print("step %d: %.1f ms, solve kernel %.1f ms, %d copies" % (k, lat[-1], solve_ms, len(copies)),
              file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    ctx.gc_release(h)
    ctx.close()

    fl = flops_per_site_update(d, w.omega)
    mean_kernel_s = float(np.mean(kms)) / 1e3
    upd_per_launch = upd / args.steps
    achieved_tflops = fl * upd_per_launch / mean_kernel_s / 1e12
    peak = PEAK_FP64_TFLOPS if w.precision == "fp64" else PEAK_FP32_TFLOPS
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
                   "orbit_seed": w.seed, "start_seed": w.start_seed},
        "site_updates_per_s": upd / wall,
        "distinct_copies_per_s": distinct / wall,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "solve_kernel_ms": float(np.mean(kms)),
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved_tflops / peak, "traffic": None,
                     "kernel": "solve_kernel", "flops_per_site_update": fl,
                     "site_updates_per_launch": upd_per_launch},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, phi, min(args.cpu_sample, n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
