"""Build libpimdb.so in place with hipcc for gfx950.

    python -m paper_2305_18025_amd.build [-v] [-j JOBS]

The fused exchange kernel is compiled once per launch variant (accumulator
rows per thread J, periodic box, mixed precision) from
``csrc/exchange_inst.hip``; the variants, the other kernels and the host
side of the ABI are compiled as separate jobs in parallel and linked into
one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libpimdb.so")
HEADERS = [os.path.join(CSRC, h) for h in ("internal.h", "common.h", "exchange.h")] + [
    os.path.join(os.path.dirname(HERE), "include", "pimdb.h")]
ARCH = os.environ.get("PIMDB_OFFLOAD_ARCH", "gfx950")

# (J rows per thread, periodic box, mixed precision) of every compiled
# exchange variant
VARIANTS = [(j, box, mixed) for j in (1, 2, 4, 8) for box in (0, 1) for mixed in (0, 1)]


def hipcc():
    cand = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def flags():
    return [
        "--offload-arch=" + ARCH,
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Wall",
        "-Wno-unused-function",
        # keep hipcc from generating packed FP32 arithmetic
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    ]


def jobs():
    """(source, extra flags, object) of every compile job."""
    out = []
    for j, box, mixed in VARIANTS:
        obj = os.path.join(CSRC, "exchange_J%d_B%d_M%d.o" % (j, box, mixed))
        out.append((os.path.join(CSRC, "exchange_inst.hip"),
                    ["-DPIMDB_J=%d" % j, "-DPIMDB_BOX=%d" % box, "-DPIMDB_MIXED=%d" % mixed], obj))
    out.append((os.path.join(CSRC, "kernels.hip"), [], os.path.join(CSRC, "kernels.o")))
    out.append((os.path.join(CSRC, "original.hip"), [], os.path.join(CSRC, "original.o")))
    out.append((os.path.join(CSRC, "pair.hip"), [], os.path.join(CSRC, "pair.o")))
    out.append((os.path.join(CSRC, "api.cpp"), [], os.path.join(CSRC, "api.o")))
    return out


def _njobs():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 4
    return max(1, min(16, n))


def build(verbose: bool = False, extra=(), njobs: int | None = None) -> str:
    """Compile every source and link libpimdb.so (always rebuilds)."""
    todo = jobs()
    t0 = time.time()

    def compile_one(job):
        src, defs, obj = job
        cmd = [hipcc()] + flags() + list(extra) + defs + ["-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        t = time.time()
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
        if verbose:
            print("  %s: %.0f s" % (os.path.basename(obj), time.time() - t), flush=True)
        return obj

    # the largest variants first, so the long jobs start early
    todo.sort(key=lambda jb: -max([int(d.split("=")[1]) for d in jb[1] if d.startswith("-DPIMDB_J")] or [0]))
    with cf.ThreadPoolExecutor(njobs or _njobs()) as ex:
        objs = list(ex.map(compile_one, todo))
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    for o in objs:
        os.remove(o)
    if verbose:
        print("built %s in %.0f s" % (SO, time.time() - t0), flush=True)
    return SO


if __name__ == "__main__":
    nj = None
    if "-j" in sys.argv:
        nj = int(sys.argv[sys.argv.index("-j") + 1])
    print(build(verbose="-v" in sys.argv, njobs=nj))
