"""Launch-shape autotuner for the exchange kernels.

The fused launch has three tunables: threads per workgroup (64..1024), the
number of particles each thread owns in the recursions (1, 2, 4, 8), and
whether (and how finely) each system's recursions are split over helper
workgroups (blocks per helper; 0 = one workgroup per recursion).  The
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


SPLITS = (4, 7, 14, 28, 56)  # blocks per helper tried for split recursions


def candidates(nmax: int, S: int = 1):
    """Launch configurations (threads, per_thread, split): whole recursions
    at every valid shape (split 0), and split recursions with each of SPLITS
    blocks per helper (threads/per_thread 0: the split kernel's own shape)
    when the batch is small enough to leave CUs idle."""
    out = []
    for per in (1, 2, 4, 8):
        for threads in (64, 128, 256, 512, 1024):
            if per >= 4 and threads > 512:
                continue
            if threads * per < nmax:
                continue
            if threads * per >= 4 * nmax and threads > 64:
                continue  # mostly idle lanes
            out.append((threads, per, 0))
    if nmax > 128 and 2 * S < 256:
        out += [(0, 0, g) for g in SPLITS]
    return out


def apply(eng, cand):
    """Set a candidate (threads, per_thread, split) on the engine; False if
    the device cannot hold it (a split plan with too many workgroups)."""
    threads, per, g = cand
    try:
        if g > 0:
            eng.set_tuning(0, 0)
            eng.set_split(g)
        else:
            eng.set_split(0)
            eng.set_tuning(threads, per)
    except RuntimeError:
        return False
    return True


def _time(eng, pos, reps: int) -> float:
    """Seconds per evaluation, HIP events on the current stream (the one the
    library enqueues on) around `reps` calls after one warm-up call."""
    F = eng.empty()
    E = torch.empty(eng.S, dtype=torch.float64, device=eng.device)
    eng.forces(pos, out=F, energy=E)
    torch.cuda.synchronize(eng.device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        eng.forces(pos, out=F, energy=E)
    e1.record()
    torch.cuda.synchronize(eng.device)
    return e0.elapsed_time(e1) * 1e-3 / reps


def autotune(eng, pos, reps: int = 3, use_cache: bool = True, verbose: bool = False, log=None):
    """Pick the fastest launch configuration for `eng` on positions `pos`,
    apply it and return (threads, per_thread, split, seconds_per_call), where
    split is the blocks per helper (0: whole recursions).  If `log` is a
    list, one dict per timed candidate is appended to it."""
    path = cache_path()
    key = cache_key(eng)
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        c = cache[key]
        cand = (c["threads"], c["per_thread"], c.get("split", 0))
        if apply(eng, cand):
            return cand + (c["seconds"],)
    best = None
    for cand in candidates(max(eng.N), eng.S):
        if not apply(eng, cand):
            continue
        sec = _time(eng, pos, reps)
        t, p = eng.tuning
        if log is not None:
            log.append({"threads": t, "per_thread": p, "split": cand[2], "ms": sec * 1e3})
        if verbose:
            print("  tune %s threads=%4d per_thread=%d split=%d  %.3f ms" % (key, t, p, cand[2], sec * 1e3),
                  flush=True)
        if best is None or sec < best[3]:
            best = (cand[0], cand[1], cand[2], sec)
    apply(eng, best[:3])
    if use_cache:
        cache[key] = {"threads": best[0], "per_thread": best[1], "split": best[2], "seconds": best[3]}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp%d" % os.getpid()
            json.dump(cache, open(tmp, "w"), indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass
    return best
