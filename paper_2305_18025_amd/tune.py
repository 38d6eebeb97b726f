"""Launch-shape autotuner for the exchange kernels.

The fused launch has two tunables: threads per workgroup (64..1024) and the
number of particles each thread owns in the recursions (1, 2, 4, 8).  The
library's built-in choice is a heuristic; this module times every valid
candidate on the device for a given batch shape and caches the fastest in a
JSON file keyed by (largest N bucket, batch size bucket, precision, box).

    from paper_2305_18025_amd import BosonicExchange
    from paper_2305_18025_amd.tune import autotune
    eng = BosonicExchange(...)
    autotune(eng, pos)            # measures (or reads the cache), applies the best
"""
from __future__ import annotations

import json
import os
import time

import torch

CACHE_ENV = "PIMDB_TUNE_CACHE"


def cache_path() -> str:
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "pimdb_tuning.json")


def _bucket(x: int) -> int:
    b = 1
    while b < x:
        b *= 2
    return b


def cache_key(eng) -> str:
    return "N%d_S%d_%s_%s" % (_bucket(max(eng.N)), _bucket(eng.S), eng.precision, "box" if eng.box > 0 else "open")


def candidates(nmax: int):
    out = []
    for per in (1, 2, 4, 8):
        for threads in (64, 128, 256, 512, 1024):
            if per >= 4 and threads > 512:
                continue
            if threads * per < nmax:
                continue
            if threads * per >= 4 * nmax and threads > 64:
                continue  # mostly idle lanes
            out.append((threads, per))
    return out


def _time(eng, pos, reps: int) -> float:
    F = eng.empty()
    E = torch.empty(eng.S, dtype=torch.float64, device=eng.device)
    eng.forces(pos, out=F, energy=E)
    torch.cuda.synchronize(eng.device)
    t0 = time.perf_counter()
    for _ in range(reps):
        eng.forces(pos, out=F, energy=E)
    torch.cuda.synchronize(eng.device)
    return (time.perf_counter() - t0) / reps


def autotune(eng, pos, reps: int = 3, use_cache: bool = True, verbose: bool = False):
    """Pick the fastest launch shape for `eng` on positions `pos`, apply it
    with eng.set_tuning and return (threads, per_thread, seconds_per_call)."""
    path = cache_path()
    key = cache_key(eng)
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        t, p = cache[key]["threads"], cache[key]["per_thread"]
        eng.set_tuning(t, p)
        return t, p, cache[key]["seconds"]
    best = None
    for (t, p) in candidates(max(eng.N)):
        eng.set_tuning(t, p)
        sec = _time(eng, pos, reps)
        if verbose:
            print("  tune %s threads=%4d per_thread=%d  %.3f ms" % (key, t, p, sec * 1e3), flush=True)
        if best is None or sec < best[2]:
            best = (t, p, sec)
    eng.set_tuning(best[0], best[1])
    if use_cache:
        cache[key] = {"threads": best[0], "per_thread": best[1], "seconds": best[2]}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp%d" % os.getpid()
            json.dump(cache, open(tmp, "w"), indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass
    return best
