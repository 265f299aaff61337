"""Build the gfx950 HIP library of the Gribov-copy enumerator in-tree.

    python -m paper_1403_0555_amd.build [--incremental]

compiles every csrc/*.hip with hipcc for gfx950 (one process per translation
unit, in parallel) into objects under _build/ and links them into
paper_1403_0555_amd/libgribov.so.  By default every unit is recompiled;
``--incremental`` recompiles only units older than a source or header.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgribov.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _headers():
    return glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(HERE, "..", "include", "*.h"))


def _compile(src: str, incremental: bool, newest_header: float):
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t >= os.path.getmtime(src) and t >= newest_header:
            return obj, None
    tmp = obj + ".tmp%d" % os.getpid()
    r = subprocess.run([HIPCC, *FLAGS, "-c", src, "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        return obj, r.stdout + r.stderr
    os.replace(tmp, obj)
    return obj, None


def build(verbose: bool = False, incremental: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    newest = max(os.path.getmtime(h) for h in _headers())
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    if verbose:
        print("hipcc %s -c <unit> (%d units, %d at a time)" % (" ".join(FLAGS), len(srcs), jobs), flush=True)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, incremental, newest), srcs))
    errors = [e for _, e in results if e]
    if errors:
        sys.stderr.write("\n".join(errors))
        raise RuntimeError("hipcc failed building %s" % LIB)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs", *[o for o, _ in results], "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed building %s" % LIB)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv[1:]))
