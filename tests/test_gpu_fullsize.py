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


def md_bound(omega_p, dt):
    """Bound on the relative excursion of the total energy in a
    velocity-Verlet run: the integrator's energy error for a mode of
    frequency w oscillates with relative size about (w dt)^2 / 8, and the
    fastest free ring-polymer mode has w = 2 omega_P; twice that estimate."""
    return (2.0 * omega_p * dt) ** 2 / 4.0


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
    eight-rows-per-thread kernel (whole recursions; the split form of the
    same systems is in the split tests): unit-density cubes, P = 8."""
    systems = [inputs.System(inputs.cube_system(4096, 8, seed=21), beta=1.0, name="open N4096"),
               inputs.System(inputs.cube_system(4033, 8, seed=22), beta=1.5, name="open N4033")]
    eng = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems], split=0)
    assert eng.tuning[:2] == (512, 8)
    pos = eng.pack([s.R for s in systems])
    F, E = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    with cf.ThreadPoolExecutor(2) as ex:
        refs = list(ex.map(_oracle_f80, systems))
    E2 = eng.energy(pos)
    mix = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems], precision="mixed", split=0)
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


def _host_vv(systems, vels, traps, dt, steps, precision="f80"):
    """Velocity Verlet on the host with oracle forces plus the harmonic trap
    (force -(m w^2 / P) r on every bead), the same update order as the GPU:
    half kick, drift, forces, half kick.  Returns positions, velocities and
    forces per system after `steps` steps."""
    out = []
    for s, V0, w in zip(systems, vels, traps):
        def force(X):
            F = oracle.alg1(X, s.beta, s.m, s.omegaP, L=s.box, precision=precision, extras=False)["F"]
            return F - (s.m * w * w / s.P) * X
        X, V = s.R.copy(), V0.copy()
        F = force(X)
        for _ in range(steps):
            V = V + 0.5 * dt / s.m * F
            X = X + dt * V
            F = force(X)
            V = V + 0.5 * dt / s.m * F
        out.append((X, V, F))
    return out


def test_velocity_verlet_multi_chunk_against_host():
    """Three velocity-Verlet steps of a batch whose systems span several of
    the 8192-element update chunks (N=700, P=16: 5 chunks; the largest member
    of the 64-system batch: ~ 25 chunks), trap omega = 1, against host
    integration with long-double oracle forces, element by element."""
    big = max(inputs.config_batch(), key=lambda x: x.N)
    systems = [inputs.System(inputs.cube_system(700, 16, seed=70), beta=0.8, m=1.3, name="N700 P16"), big]
    vels = [inputs.initial_velocities(s.N, s.P, s.beta, s.m, seed=71 + i) for i, s in enumerate(systems)]
    dt, w = 0.01, 1.0
    eng = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems], trap=w)
    assert all(3 * s.P * s.N > 4 * 8192 for s in systems)
    md = VelocityVerlet(eng, eng.pack([s.R for s in systems]), eng.pack(vels), dt)
    md.step(3)
    torch.cuda.synchronize()
    assert eng.status() == 0
    with cf.ThreadPoolExecutor(2) as ex:
        refs = list(ex.map(lambda i: _host_vv([systems[i]], [vels[i]], [w], dt, 3)[0], range(2)))
    for i, (s, (X, V, F)) in enumerate(zip(systems, refs)):
        ex_ = np.abs(eng.unpack(md.pos, i) - X).max() / np.abs(X).max()
        ev = np.abs(eng.unpack(md.vel, i) - V).max() / np.abs(V).max()
        ef = np.abs(eng.unpack(md.forces, i) - F).max() / np.abs(F).max()
        print("%s (%d elements): positions %.2e velocities %.2e forces %.2e" % (s.name, 3 * s.P * s.N, ex_, ev, ef))
        assert ex_ <= TOL64 and ev <= TOL64 and ef <= TOL64


def test_large_system_mixed_md_two_steps_against_host():
    """The periodic N=4096, P=64 system in the mixed mode (FP32 pair lengths,
    FP64 recursions), two velocity-Verlet steps (dt = 0.01, no trap) against
    host integration with long-double oracle forces: forces within the
    mixed tolerance, positions and velocities well inside it."""
    s = inputs.config_large()
    V0 = inputs.initial_velocities(s.N, s.P, s.beta, s.m, seed=55)
    eng = BosonicExchange(s.N, s.P, s.beta, s.m, s.omegaP, box=s.box, precision="mixed")
    md = VelocityVerlet(eng, eng.pack(s.R), eng.pack(V0), 0.01)
    md.step(2)
    torch.cuda.synchronize()
    assert eng.status() == 0
    X, V, F = _host_vv([s], [V0], [0.0], 0.01, 2)[0]
    ex_ = np.abs(eng.unpack(md.pos, 0) - X).max() / np.abs(X).max()
    ev = np.abs(eng.unpack(md.vel, 0) - V).max() / np.abs(V).max()
    ef = np.abs(eng.unpack(md.forces, 0) - F).max() / np.abs(F).max()
    print("N=4096 P=64 periodic mixed, 2 steps: positions %.2e velocities %.2e forces %.2e" % (ex_, ev, ef))
    assert ef <= TOLMIX and ev <= TOLMIX and ex_ <= TOLMIX


def _total_energy(md):
    return (md.kinetic() + md.energy).double().cpu().numpy()


def test_large_system_mixed_md_200_steps():
    """200 graph-captured velocity-Verlet steps (dt = 0.01) of the periodic
    N=4096, P=64 system in the mixed mode: finite, status clear, and the total
    energy (kinetic + V^[1,N]) stays within md_bound of its start."""
    s = inputs.config_large()
    eng = BosonicExchange(s.N, s.P, s.beta, s.m, s.omegaP, box=s.box, precision="mixed")
    pos = eng.pack(s.R)
    vel = eng.pack(inputs.initial_velocities(s.N, s.P, s.beta, s.m, seed=55))
    md = VelocityVerlet(eng, pos, vel, 0.01)
    e0 = _total_energy(md)
    md.capture(steps_per_replay=50)
    worst = 0.0
    for _ in range(4):
        md.replay(1)
        torch.cuda.synchronize()
        worst = max(worst, float(np.abs(_total_energy(md) - e0).max() / np.abs(e0).max()))
    assert eng.status() == 0
    print("N=4096 P=64 mixed: largest |E(t) - E(0)| / |E(0)| over 200 steps = %.2e (bound %.2e)"
          % (worst, md_bound(s.omegaP, 0.01)))
    assert np.isfinite(worst) and worst < md_bound(s.omegaP, 0.01)


def test_uneven_batch_md_1000_steps():
    """The 64-system batch with a harmonic trap (omega = 1), dt = 0.01 and
    Maxwell-Boltzmann initial velocities: 1000 velocity-Verlet steps replayed
    from a HIP graph (100 steps per replay); every system stays finite, the
    device status stays clear and each system's total energy (kinetic +
    V^[1,N] + trap) stays within md_bound of its start, sampled every 100
    steps."""
    systems = inputs.config_batch()
    eng = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems], trap=1.0)
    pos = eng.pack([s.R for s in systems])
    vel = eng.pack([inputs.initial_velocities(s.N, s.P, s.beta, s.m, seed=100 + i) for i, s in enumerate(systems)])
    md = VelocityVerlet(eng, pos, vel, 0.01)
    e0 = _total_energy(md)
    md.capture(steps_per_replay=100)
    worst = np.zeros(len(systems))
    for _ in range(10):
        md.replay(1)
        torch.cuda.synchronize()
        worst = np.maximum(worst, np.abs(_total_energy(md) - e0) / np.abs(e0))
    assert eng.status() == 0
    assert torch.isfinite(md.pos).all() and torch.isfinite(md.energy).all()
    bound = np.array([md_bound(s.omegaP, 0.01) for s in systems])
    i = int(np.argmax(worst / bound))
    print("64 systems, 1000 steps: largest relative energy excursion %.2e of its bound %.2e (system %d, %s)"
          % (worst[i], bound[i], i, systems[i].name))
    assert (worst < bound).all()
