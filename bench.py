#!/usr/bin/env python3
"""Benchmark: bosonic exchange energy + force evaluations per second at
N = 1024 particles, P = 32 beads on one MI355X.

A step is one evaluation of the whole exchange path (interior springs,
forward and backward recursions, connection-probability forces, energies)
for a batch of B independent N=1024, P=32 systems, with positions already
resident in HBM.  The evaluations run from a HIP graph that holds several
consecutive evaluations (as an MD loop captures several steps), replayed
until exactly `steps` evaluations are timed.  `value` is B * steps / seconds.

Also reported (same JSON line): the plain one-system-per-call path without a
graph, a batch-size sweep, the mixed-precision variant, accuracy against the
CPU oracle, the roofline of the fused kernel measured with HIP events, and
the CPU oracle's own throughput on the host cores (a bounded sample).

    python bench.py [--steps K] [--warmup W] [--batch B]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exchange E+F evals/sec at N=1024,P=32 (batched vs plain, 1 GPU)"
N_HEAD, P_HEAD, BETA = 1024, 32, 1.0
PEAK_FP64 = 78.6e12  # MI355X FP64 vector peak: 256 CU * 4 SIMD * 16 lanes * 2 flop * 2.4 GHz
# Algorithmic work of one evaluation: the method's O(N^2) part is three
# passes of M = N(N+1)/2 exponentials (the forward potentials, the backward
# potentials and the connection probabilities), each a double-precision
# exponential of about 16 FP64 operations (range reduction and a
# polynomial) -- 25.2 MFLOP at N = 1024.  The fused kernels here reuse the
# two recursions' terms for the probabilities (two passes), so this counts
# more work than they issue.
EXP_FLOPS = 16


def flops_per_eval(N: int) -> float:
    return 3.0 * (N * (N + 1) / 2) * EXP_FLOPS


def systems(B, seed0=3, variant="gaussian"):
    from paper_2305_18025_amd import inputs
    if variant == "gaussian":
        return [inputs.gaussian_system(N_HEAD, P_HEAD, seed=seed0 + i) for i in range(B)]
    return [inputs.cube_system(N_HEAD, P_HEAD, seed=seed0 + i) for i in range(B)]


def make_engine(B, precision="fp64", tuning=None):
    from paper_2305_18025_amd import BosonicExchange
    kw = {}
    if tuning:
        kw = dict(threads=tuning[0], per_thread=tuning[1])
    return BosonicExchange([N_HEAD] * B, [P_HEAD] * B, [BETA] * B, 1.0, precision=precision, **kw)


# Evaluations captured in one graph at most: a single-evaluation graph pays
# the graph launch between every two evaluations (0.409 against 0.353 ms
# per evaluation of the 256-system batch with ten per graph)
EVALS_PER_GRAPH = 10
# Untimed evaluations before a graph is timed, at least: the device reaches
# its steady clock after some tens of milliseconds of continuous work (the
# 256-system batch measures 0.38 ms per evaluation after 5, 0.36 after 50)
MIN_WARMUP_EVALS = 50


def evals_per_graph(steps, most=EVALS_PER_GRAPH):
    """The largest divisor of `steps` not above `most`, so that whole
    replays time exactly `steps` evaluations."""
    for n in range(min(most, steps), 0, -1):
        if steps % n == 0:
            return n
    return 1


def warmup_replays(steps, warmup):
    """Untimed replays of a graph of evals_per_graph(steps) evaluations."""
    n = evals_per_graph(steps)
    return (max(warmup, MIN_WARMUP_EVALS) + n - 1) // n


def time_graph(eng, pos, steps, warmup):
    """Capture n = evals_per_graph(steps) consecutive exchange_forces calls
    in one graph; replay it for at least max(warmup, MIN_WARMUP_EVALS)
    untimed evaluations, then for exactly `steps` timed ones.  Returns (wall
    seconds for the `steps` evaluations, event-timed ms per evaluation,
    (F, E))."""
    import torch
    n = evals_per_graph(steps)
    F = eng.empty()
    E = torch.empty(eng.S, dtype=torch.float64, device=eng.device)
    eng.forces(pos, out=F, energy=E)  # eager warm-up before capture
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            for _ in range(n):
                eng.forces(pos, out=F, energy=E)
    torch.cuda.current_stream().wait_stream(side)
    for _ in range(warmup_replays(steps, warmup)):
        g.replay()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps // n):
        g.replay()
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / steps, (F, E)


def accuracy(eng, F, E, R_list, precision="f80", which=(0,)):
    """Largest relative energy error and norm-wise force error
    (max|dF| / max|F|) over the systems `which`, against the oracle, plus
    per-component statistics of the force error."""
    import numpy as np
    import oracle
    from paper_2305_18025_amd.inputs import omega_p
    ee = fe = 0.0
    comp = {"x": 0.0, "y": 0.0, "z": 0.0}
    elem = []
    for s in which:
        o = oracle.alg1(R_list[s], BETA, 1.0, omega_p(P_HEAD, BETA), precision=precision, extras=False)
        Fg = eng.unpack(F, s)
        d = np.abs(Fg - o["F"])
        ee = max(ee, abs(float(E[s]) - o["V"]) / abs(o["V"]))
        fe = max(fe, float(d.max() / np.abs(o["F"]).max()))
        for c, name in enumerate("xyz"):
            comp[name] = max(comp[name], float(d[..., c].max() / np.abs(o["F"][..., c]).max()))
        big = np.abs(o["F"]) > 1e-3 * np.abs(o["F"]).max()
        elem.append(d[big] / np.abs(o["F"][big]))
    elem = np.concatenate(elem)
    stats = {"max_abs_err_over_max_abs_F_by_component": comp,
             "elementwise_rel_err_median": float(np.median(elem)),
             "elementwise_rel_err_p99": float(np.quantile(elem, 0.99)),
             "elementwise_rel_err_max": float(elem.max()),
             "elementwise_note": "|dF_i| / |F_i| over components with |F_i| > 1e-3 max|F|"}
    return ee, fe, stats


def kernel_times(eng, pos, reps, lead=3):
    """Mean durations (ms) of the exchange and finalize launches over `reps`
    eager evaluations, from HIP events the library records on its stream.
    Each timed evaluation follows `lead` others issued back to back, so it
    starts on a busy device, as the evaluations of a graph do (one issued
    after the host has waited runs about 10% longer)."""
    import torch
    F = eng.empty()
    E = torch.empty(eng.S, dtype=torch.float64, device=eng.device)
    eng.set_timing(True)
    ex = fi = 0.0
    for _ in range(reps):
        for _ in range(lead + 1):
            eng.forces(pos, out=F, energy=E)
        a, b = eng.last_timing()
        ex += a
        fi += b
    eng.set_timing(False)
    return ex / reps, fi / reps


def time_calls(fn, reps):
    """Average ms of fn() over reps calls, HIP events on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def extra_workloads(steps):
    """The other configurations, measured as context: the 64-system uneven
    batch (one evaluation and one velocity-Verlet step with the trap, both
    graph-replayed), the periodic N=4096, P=64 system (evaluation and MD
    step), and the endpoint-spring table export."""
    import torch
    from paper_2305_18025_amd import BosonicExchange, VelocityVerlet, inputs
    out = {}
    systems = inputs.config_batch()
    eng = BosonicExchange([x.N for x in systems], [x.P for x in systems], [x.beta for x in systems],
                          [x.m for x in systems], [x.omegaP for x in systems], trap=1.0)
    pos = eng.pack([x.R for x in systems])
    w, ms, _ = time_graph(eng, pos, steps, 2)
    vel = eng.pack([inputs.initial_velocities(x.N, x.P, x.beta, x.m, seed=100 + i) for i, x in enumerate(systems)])
    md = VelocityVerlet(eng, pos.clone(), vel, 0.01)
    md.capture(steps_per_replay=10)
    md_ms = time_calls(lambda: md.replay(1), max(2, steps // 10)) / 10
    out["uneven_batch"] = {"systems": len(systems), "N_range": [min(x.N for x in systems), max(x.N for x in systems)],
                           "evals_per_s": len(systems) / (ms * 1e-3), "ms_per_eval": ms,
                           "md_ms_per_step": md_ms, "launch_shape": list(eng.tuning)}
    del eng, pos, vel, md
    x = inputs.config_large()
    eng = BosonicExchange(x.N, x.P, x.beta, x.m, x.omegaP, box=x.box)
    pos = eng.pack(x.R)
    F = eng.empty()
    E = torch.empty(1, dtype=torch.float64, device=eng.device)
    ms = time_calls(lambda: eng.forces(pos, out=F, energy=E), steps)
    vel = eng.pack(inputs.initial_velocities(x.N, x.P, x.beta, x.m, seed=55))
    md = VelocityVerlet(eng, pos.clone(), vel, 0.001)
    md.capture(steps_per_replay=10)
    md_ms = time_calls(lambda: md.replay(1), max(2, steps // 10)) / 10
    out["large_periodic"] = {"N": x.N, "P": x.P, "box": x.box, "ms_per_eval": ms, "evals_per_s": 1e3 / ms,
                             "ns_per_recursion_step": ms * 1e6 / x.N, "md_ms_per_step": md_ms,
                             "launch_shape": list(eng.tuning)}
    # endpoint-spring table s(v,u), u <= v: M values written per call
    tab = {}
    for n, s_ in ((N_HEAD, None), (x.N, x)):
        if s_ is None:
            e2 = BosonicExchange(n, P_HEAD, BETA)
            p2 = e2.pack(inputs.gaussian_system(n, P_HEAD, seed=3))
        else:
            e2, p2 = eng, pos
        M = n * (n + 1) // 2
        for as_float in (False, True):
            buf = torch.empty(M, dtype=torch.float32 if as_float else torch.float64, device=e2.device)
            t = time_calls(lambda: e2.endpoint_springs(p2, 0, as_float=as_float, out=buf), steps)
            nbytes = M * (4 if as_float else 8) + 2 * 3 * n * 8
            tab["N%d_%s" % (n, "f32" if as_float else "f64")] = {"ms": t, "GB_per_s": nbytes / (t * 1e-3) / 1e9,
                                                                  "frac_of_8TBs": nbytes / (t * 1e-3) / 8e12}
    out["endpoint_table"] = tab
    return out


def fast_vs_original(sizes=(32, 64, 128, 256, 512, 1024), P=32, beta=1.0, trap=1.0):
    """Time per evaluation (energy and forces of one system, HIP events over
    the calls) of the quadratic algorithm and of the original cubic one on
    the same GPU, for cold trapped systems of N particles with P = 32 beads
    (the scaling benchmark's setting), and the log-log slopes."""
    import numpy as np
    import torch
    from paper_2305_18025_amd import BosonicExchange, inputs
    rows = []
    for n in sizes:
        x = inputs.System(inputs.gaussian_system(n, P, seed=n), beta=beta)
        t = {}
        for alg in ("fast", "original"):
            eng = BosonicExchange(n, P, beta, trap=trap, algorithm=alg)
            pos = eng.pack(x.R)
            F = eng.empty()
            E = torch.empty(1, dtype=torch.float64, device=eng.device)
            eng.forces(pos, out=F, energy=E)
            torch.cuda.synchronize()
            reps = 50 if alg == "fast" else max(3, min(50, int(200 * (64.0 / n) ** 2)))
            t[alg] = time_calls(lambda: eng.forces(pos, out=F, energy=E), reps)
            if eng.status() != 0:
                raise RuntimeError("device status set in the %s algorithm at N=%d" % (alg, n))
            del eng, pos, F, E
            torch.cuda.empty_cache()
        rows.append({"N": n, "fast_ms": t["fast"], "original_ms": t["original"],
                     "speedup": t["original"] / t["fast"]})
    lg = lambda key: np.polyfit(np.log([r["N"] for r in rows]), np.log([r[key] for r in rows]), 1)[0]
    tail = rows[-3:]
    lgt = lambda key: np.polyfit(np.log([r["N"] for r in tail]), np.log([r[key] for r in tail]), 1)[0]
    return {"P": P, "beta": beta, "trap": trap, "rows": rows,
            "loglog_slope_all": {"fast": lg("fast_ms"), "original": lg("original_ms"), "speedup": lg("speedup")},
            "loglog_slope_last3": {"fast": lgt("fast_ms"), "original": lgt("original_ms"),
                                   "speedup": lgt("speedup")},
            "description": "one system per call, no graph; the original algorithm's cycle energies by "
                           "their defining sum, its forces by the per-bead derivative recurrence"}


# Algorithmic work of the scaled pair interaction per unordered pair: the
# displacement and its square (3 + 5 flops), the exponent (1), the
# exponential (EXP_FLOPS), the energy (1) and the two beads' forces (2 x 3
# fused multiply-adds).
PAIR_FLOPS = 3 + 5 + 1 + EXP_FLOPS + 1 + 12


def pair_interaction(steps=10, g=3.0, sigma=0.5):
    """The scaled Gaussian pair interaction alone (pimdb_pair_forces) on the
    periodic N=4096, P=64 system and on the headline batch, HIP events over
    the calls; its ALU roofline by the unordered-pair count."""
    import torch
    from paper_2305_18025_amd import BosonicExchange, inputs
    out = {}
    x = inputs.config_large()
    head = [inputs.System(R, beta=BETA) for R in systems(256)]
    cases = [("large_periodic", [x], x.box), ("headline_batch_256", head, 0.0)]
    for name, sys_, box in cases:
        eng = BosonicExchange([q.N for q in sys_], [q.P for q in sys_], [q.beta for q in sys_],
                              [q.m for q in sys_], [q.omegaP for q in sys_], box=box, pair=(g, sigma))
        pos = eng.pack([q.R for q in sys_])
        F = eng.empty()
        E = torch.empty(eng.S, dtype=torch.float64, device=eng.device)
        ms = time_calls(lambda: eng.pair_forces(pos, out=F, energy=E), steps)
        if eng.status() != 0:
            raise RuntimeError("device status set in the pair interaction")
        pairs = sum(q.P * q.N * (q.N - 1) / 2 for q in sys_)
        fl = pairs * PAIR_FLOPS
        out[name] = {"systems": len(sys_), "N": sys_[0].N, "P": sys_[0].P, "box": box, "ms_per_call": ms,
                     "unordered_pairs": pairs, "pairs_per_s": pairs / (ms * 1e-3),
                     "tflops": fl / (ms * 1e-3) / 1e12, "frac_of_fp64_peak": fl / (ms * 1e-3) / PEAK_FP64}
        del eng, pos, F, E
        torch.cuda.empty_cache()
    out["flops_per_pair"] = PAIR_FLOPS
    out["U"] = {"g": g, "sigma": sigma, "form": "g exp(-r^2 / (2 sigma^2)), caller-parameterised"}
    return out


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(seconds, max_threads=16):
    """The FP64 C oracle (as it stands) on the host cores: single-thread
    median latency of the plain N=256 and the headline N=1024 evaluations,
    then independent N=1024, P=32 evaluations (energy + forces) in a thread
    pool for about `seconds` of wall time.  The pool is capped at 16 threads,
    the CPU share of one GPU on the measurement boxes."""
    import concurrent.futures as cf
    import statistics
    import oracle
    from paper_2305_18025_amd import inputs
    from paper_2305_18025_amd.inputs import gaussian_system, omega_p
    model, avail = host_info()
    cores = max(1, min(max_threads, avail))
    oracle.build(force=False)
    single = {}
    for name, sy in (("N256_P32_cube", inputs.config_plain()), ("N1024_P32_gaussian", inputs.config_headline())):
        ts = []
        for _ in range(7):
            t0 = time.perf_counter()
            oracle.alg1(sy.R, sy.beta, sy.m, sy.omegaP, precision="f64", extras=False)
            ts.append(time.perf_counter() - t0)
        single[name] = {"median_ms": statistics.median(ts) * 1e3, "evaluations": len(ts)}
    Rs = [gaussian_system(N_HEAD, P_HEAD, seed=1000 + i) for i in range(cores)]
    w = omega_p(P_HEAD, BETA)
    deadline = time.perf_counter() + seconds

    def worker(i):
        n = 0
        while time.perf_counter() < deadline:
            oracle.alg1(Rs[i], BETA, 1.0, w, precision="f64", extras=False)
            n += 1
        return n

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        counts = list(ex.map(worker, range(cores)))
    dt = time.perf_counter() - t0
    total = sum(counts)
    return {"value": total / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": "%d evaluations (energy+forces, FP64 oracle in C, N=1024 P=32 Gaussian) "
                      "on %d host threads in %.1f s" % (total, cores, dt),
            "host_cpu": model, "host_cores_available": avail, "threads_used": cores,
            "single_thread_latency": single}


def device_sources_sha1():
    from paper_2305_18025_amd.profiling import device_sources_sha1 as f
    return f()


def traffic_record(batch):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current device sources and batch size."""
    path = os.path.join(ROOT, "profiles", "exchange_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("device_sources_sha1") != device_sources_sha1() or rec.get("batch") != batch:
        return None
    return rec.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--sweep", default="1,8,64,256,512")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline and plain only")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's built-in launch shape instead of timing the candidates")
    ap.add_argument("--plain-calls", type=int, default=1000)
    ap.add_argument("--profile-run", nargs="?", const="headline", default=None,
                    choices=("headline", "original", "pair"),
                    help="only run one workload for rocprofv3: the headline launch (graph replays, then "
                         "a 256 MiB copy as the traffic calibration kernel), the original algorithm at "
                         "N=1024, P=32 (steps calls), or the pair interaction of the periodic N=4096, "
                         "P=64 system (steps calls)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this implementation runs on one GPU (one MI355X per box); "
              "--gpus %d is not supported" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_18025_amd.tune import autotune

    if args.profile_run in ("original", "pair"):
        from paper_2305_18025_amd import BosonicExchange, inputs
        if args.profile_run == "original":
            x = inputs.System(inputs.gaussian_system(N_HEAD, P_HEAD, seed=3), beta=BETA)
            eng = BosonicExchange(x.N, x.P, x.beta, trap=1.0, algorithm="original")
        else:
            x = inputs.config_large()
            eng = BosonicExchange(x.N, x.P, x.beta, x.m, x.omegaP, box=x.box, pair=(3.0, 0.5))
        pos = eng.pack(x.R)
        F = eng.empty()
        E = torch.empty(1, dtype=torch.float64, device=eng.device)
        run = (lambda: eng.forces(pos, out=F, energy=E)) if args.profile_run == "original" else \
            (lambda: eng.pair_forces(pos, out=F, energy=E))
        for _ in range(args.warmup + args.steps):
            run()
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": args.profile_run, "calls": args.warmup + args.steps,
                          "status": eng.status()}))
        return

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B = args.batch
    Rb = systems(B)

    # headline: batched, graph-captured, launch shape from the autotuner
    eng = make_engine(B)
    pos = eng.pack(Rb)
    tune_log = None
    if args.no_autotune or args.profile_run:
        tuned = eng.tuning
    else:
        tune_log = []
        tuned = autotune(eng, pos, reps=3, use_cache=False, log=tune_log)
    wall, ms_launch, (F, E) = time_graph(eng, pos, args.steps, args.warmup)
    if args.profile_run:
        src = torch.empty(256 << 20, dtype=torch.uint8, device=eng.device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "batch": B, "steps": args.steps, "warmup": args.warmup,
                          "evals_per_graph": evals_per_graph(args.steps),
                          "launch_shape": list(tuned[:2]), "calibration_copy_bytes": 256 << 20}))
        return
    value = B * args.steps / wall
    torch.cuda.synchronize()
    status = eng.status()
    # the dominant kernel alone: HIP events around the exchange launch
    ms_exchange, ms_finalize = kernel_times(eng, pos, max(10, args.steps))

    # plain: one system per call, no graph, library launch shape; HIP events
    # on the library's stream (torch's current stream) over the calls
    eng1 = make_engine(1)
    pos1 = eng1.pack(Rb[0])
    F1 = eng1.empty()
    E1 = torch.empty(1, dtype=torch.float64, device=eng1.device)
    ms_plain = time_calls(lambda: eng1.forces(pos1, out=F1, energy=E1), args.plain_calls)
    ms_plain_ex, ms_plain_fin = kernel_times(eng1, pos1, 20)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "bosonic exchange energy+forces, batch of %d systems, N=1024, P=32, beta=1, m=1, "
                        "omega_P=sqrt(P)/beta; centroids N(0,1), beads centroid+N(0,0.3^2); one evaluation "
                        "(exchange + finalize launches) per step, %d steps per HIP-graph replay"
                        % (B, evals_per_graph(args.steps)),
            "N": N_HEAD, "P": P_HEAD, "batch": B, "precision": "fp64", "graph": True,
            "evals_per_graph": evals_per_graph(args.steps),
            "warmup_evals": warmup_replays(args.steps, args.warmup) * evals_per_graph(args.steps),
            "launch_shape": {"threads": tuned[0], "per_thread": tuned[1]},
        },
        "plain": {"value": 1e3 / ms_plain, "unit": "evals/s", "ms_per_eval": ms_plain, "calls": args.plain_calls,
                  "exchange_kernel_ms": ms_plain_ex, "finalize_kernel_ms": ms_plain_fin,
                  "ns_per_recursion_step": ms_plain * 1e6 / N_HEAD,
                  "description": "one system per call, no graph, HIP events over the calls"},
        "batched_over_plain": value * ms_plain * 1e-3,
        "device_status": status,
    }
    if tune_log is not None:
        out["autotune"] = tune_log
    flops = B * flops_per_eval(N_HEAD)
    achieved = flops / (ms_exchange * 1e-3)
    out["roofline"] = {
        "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64, "traffic": traffic_record(B),
        "kernel": "pimdb::k_exchange%s<%d, false, false> (fused springs + recursions)"
                  % ("_wide" if tuned[1] >= 4 else "", tuned[1]),
        "ms_per_launch_hip_events": ms_exchange,
        "finalize_ms_hip_events": ms_finalize,
        "graph_ms_per_eval": ms_launch,
        "flops_per_launch": flops,
        "flops_per_eval": flops_per_eval(N_HEAD),
        "flop_model": "3 passes of N(N+1)/2 FP64 exponentials at %d flops each" % EXP_FLOPS,
        "device_sources_sha1": device_sources_sha1(),
    }

    if not args.quick:
        ee, fe, st = accuracy(eng, F, E, Rb, "f80", which=(0, B - 1))
        out["accuracy_vs_oracle_f80"] = {"energy_rel": ee, "forces_rel_max": fe, "tolerance": 1e-10,
                                         "forces_per_component": st}
        sweep = {}
        sub = max(EVALS_PER_GRAPH, args.steps // (2 * EVALS_PER_GRAPH) * EVALS_PER_GRAPH)
        for b in [int(x) for x in args.sweep.split(",") if x]:
            e_b = make_engine(b)
            p_b = e_b.pack(Rb[:b] if b <= B else systems(b))
            w_b, ms_b, _ = time_graph(e_b, p_b, sub, 2)
            sweep[str(b)] = {"evals_per_s": b * sub / w_b, "ms_per_eval": ms_b,
                             "launch_shape": list(e_b.tuning)}
            del e_b, p_b
        out["batch_sweep"] = sweep
        em = make_engine(B, precision="mixed", tuning=tuned[:2])
        pm = em.pack(Rb)
        w_m, ms_m, (Fm, Em) = time_graph(em, pm, sub, 2)
        eem, fem, _ = accuracy(em, Fm, Em, Rb, "f80", which=(0,))
        out["mixed"] = {"evals_per_s": B * sub / w_m, "energy_rel": eem,
                        "forces_rel_max": fem, "tolerance": 1e-5,
                        "description": "FP32 compensated endpoint-spring lengths, FP64 elsewhere"}
        del em, pm
        # distinguishable-particle reference cost (same batch, same launch)
        Fd = eng.empty()
        Ed = torch.empty(B, dtype=torch.float64, device=eng.device)
        eng.distinguishable(pos, Fd, Ed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            eng.distinguishable(pos, Fd, Ed)
        torch.cuda.synchronize()
        sec_d = (time.perf_counter() - t0) / args.steps
        spring_bytes = 2 * pos.numel() * 8  # every bead read and written once
        out["distinguishable"] = {"evals_per_s": B / sec_d,
                                  "description": "ring-polymer springs without exchange, same batch",
                                  "springs_TB_per_s": spring_bytes / sec_d / 1e12,
                                  "springs_frac_of_8TBs": spring_bytes / sec_d / 8e12}
        out.update(extra_workloads(args.steps))
        out["fast_vs_original"] = fast_vs_original()
        out["pair_interaction"] = pair_interaction()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
