"""GPU parity at the full workload sizes: the 64-system uneven batch
(N up to 2048, P in {16, 32, 64}, beta in [0.5, 2]), the periodic
N=4096, P=64 system and open systems at the largest accepted N, against the
long-double oracle."""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2305_18025_amd import BosonicExchange, VelocityVerlet, inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOLMIX = 1e-5


def _oracle_f80(s):
    return oracle.alg1(s.R, s.beta, s.m, s.omegaP, L=s.box, precision="f80", extras=False)


def _threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 4


def test_open_maximum_size():
    """Open boundaries at the largest N the ABI accepts (4096, exactly 64
    blocks) and a ragged neighbour (4033 = 63 blocks + 1), one batch, the
    eight-rows-per-thread kernel: unit-density cubes, P = 8."""
    systems = [inputs.System(inputs.cube_system(4096, 8, seed=21), beta=1.0, name="open N4096"),
               inputs.System(inputs.cube_system(4033, 8, seed=22), beta=1.5, name="open N4033")]
    eng = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems])
    assert eng.tuning[:2] == (512, 8)
    pos = eng.pack([s.R for s in systems])
    F, E = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    with cf.ThreadPoolExecutor(2) as ex:
        refs = list(ex.map(_oracle_f80, systems))
    E2 = eng.energy(pos)
    mix = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems], precision="mixed")
    Fm, Em = mix.forces(pos)
    torch.cuda.synchronize()
    assert mix.status() == 0
    for i, (s, o) in enumerate(zip(systems, refs)):
        ee = abs(float(E[i]) - o["V"]) / abs(o["V"])
        fe = float(np.abs(eng.unpack(F, i) - o["F"]).max() / np.abs(o["F"]).max())
        ee2 = abs(float(E2[i]) - o["V"]) / abs(o["V"])
        eem = abs(float(Em[i]) - o["V"]) / abs(o["V"])
        fem = float(np.abs(mix.unpack(Fm, i) - o["F"]).max() / np.abs(o["F"]).max())
        print("%s: energy %.2e forces %.2e energy-only %.2e; mixed energy %.2e forces %.2e"
              % (s.name, ee, fe, ee2, eem, fem))
        assert ee <= TOL64 and fe <= TOL64 and ee2 <= TOL64
        assert eem <= TOLMIX and fem <= TOLMIX


def test_uneven_batch_of_64_full_size():
    systems = inputs.config_batch()
    eng = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems])
    pos = eng.pack([s.R for s in systems])
    F, E = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    with cf.ThreadPoolExecutor(_threads()) as ex:
        refs = list(ex.map(_oracle_f80, systems))
    worst = (0.0, 0.0)
    for i, (s, o) in enumerate(zip(systems, refs)):
        ee = abs(float(E[i]) - o["V"]) / abs(o["V"])
        fe = float(np.abs(eng.unpack(F, i) - o["F"]).max() / np.abs(o["F"]).max())
        worst = (max(worst[0], ee), max(worst[1], fe))
        assert ee <= TOL64 and fe <= TOL64, (i, s.name, ee, fe)
    print("64 systems: worst energy %.2e forces %.2e" % worst)


def test_periodic_large_system_full_size():
    s = inputs.config_large()
    eng = BosonicExchange(s.N, s.P, s.beta, s.m, s.omegaP, box=s.box)
    pos = eng.pack(s.R)
    F, E = eng.forces(pos)
    o = _oracle_f80(s)
    ee = abs(float(E[0]) - o["V"]) / abs(o["V"])
    fe = float(np.abs(eng.unpack(F, 0) - o["F"]).max() / np.abs(o["F"]).max())
    print("N=4096 P=64 periodic: energy %.2e forces %.2e" % (ee, fe))
    assert ee <= TOL64 and fe <= TOL64
    Fm, Em = BosonicExchange(s.N, s.P, s.beta, s.m, s.omegaP, box=s.box, precision="mixed").forces(pos)
    eem = abs(float(Em[0]) - o["V"]) / abs(o["V"])
    fem = float(np.abs(eng.unpack(Fm, 0) - o["F"]).max() / np.abs(o["F"]).max())
    print("  mixed: energy %.2e forces %.2e" % (eem, fem))
    assert eem <= TOLMIX and fem <= TOLMIX


def test_large_system_md_graph_runs():
    """200 graph-captured MD steps of the periodic N=4096, P=64 system stay
    finite and conserve the total energy to a loose bound."""
    s = inputs.config_large()
    eng = BosonicExchange(s.N, s.P, s.beta, s.m, s.omegaP, box=s.box)
    pos = eng.pack(s.R)
    vel = eng.pack(inputs.initial_velocities(s.N, s.P, s.beta, s.m, seed=55))
    md = VelocityVerlet(eng, pos, vel, 0.001)
    e0 = float(md.kinetic()[0] + md.energy[0])
    md.capture(steps_per_replay=50)
    md.replay(4)
    torch.cuda.synchronize()
    assert eng.status() == 0
    e1 = float(md.kinetic()[0] + md.energy[0])
    assert np.isfinite(e1) and abs(e1 - e0) < 1e-3 * abs(e0)


def test_uneven_batch_md_1000_steps():
    """The 64-system batch with a harmonic trap (omega = 1), dt = 0.01 and
    Maxwell-Boltzmann initial velocities: 1000 velocity-Verlet steps replayed
    from a HIP graph (100 steps per replay); every system stays finite and the
    device status stays clear."""
    systems = inputs.config_batch()
    eng = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems], trap=1.0)
    pos = eng.pack([s.R for s in systems])
    vel = eng.pack([inputs.initial_velocities(s.N, s.P, s.beta, s.m, seed=100 + i) for i, s in enumerate(systems)])
    md = VelocityVerlet(eng, pos, vel, 0.01)
    md.capture(steps_per_replay=100)
    md.replay(10)
    torch.cuda.synchronize()
    assert eng.status() == 0
    assert torch.isfinite(md.pos).all() and torch.isfinite(md.energy).all()
