"""GPU: the scaled Gaussian pair interaction (1/P) sum_j sum_{a<b} U, alone
and added to the exchange forces and energies, against the CPU pair oracle
(oracle/pair.py) and the long-double exchange oracle, in every entry that
writes forces or energies."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from oracle.pair import pair_gaussian, pair_gaussian_at
from paper_2305_18025_amd import BosonicExchange, _lib, exchange_potential, inputs
from paper_2305_18025_amd.inputs import System, cube_system, gaussian_system

pytestmark = pytest.mark.gpu

TOL = 1e-10
G, SIG = 3.0, 0.5  # a repulsive Gaussian of the caller's choosing


def _engine(systems, **kw):
    eng = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems], **kw)
    return eng, eng.pack([s.R for s in systems])


def _rel(a, b):
    return abs(a - b) / abs(b)


def _frel(F, ref):
    return float(np.abs(F - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("N,P,box", [(1, 2, 0.0), (2, 3, 0.0), (7, 4, 2.0), (65, 5, 0.0), (300, 8, 6.0),
                                     (513, 2, 0.0)])
def test_pair_alone_matches_oracle(N, P, box):
    """Ragged particle counts around the 64/128/256-particle workgroups and
    the 256-particle LDS tiles, one particle (no pairs), periodic boxes."""
    R = cube_system(N, P, seed=N, side=box if box else None)
    s = System(R, beta=1.0, box=box)
    eng, pos = _engine([s], box=box, pair=(G, SIG))
    F, E = eng.pair_forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    Eo, Fo = pair_gaussian(R, G, SIG, L=box)
    Fg = eng.unpack(F, 0)
    if N == 1:
        assert float(E[0]) == 0.0 and np.abs(Fg).max() == 0.0
        return
    print("  N=%d P=%d: energy %.2e forces %.2e" % (N, P, _rel(float(E[0]), Eo), _frel(Fg, Fo)))
    assert _rel(float(E[0]), Eo) <= 1e-12
    assert _frel(Fg, Fo) <= 1e-12


def test_pair_headline_size():
    """N = 1024, P = 32 (the headline system) against the whole double sum."""
    s = inputs.config_headline()
    eng, pos = _engine([s], pair=(G, SIG))
    F, E = eng.pair_forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    Eo, Fo = pair_gaussian(s.R, G, SIG)
    assert _rel(float(E[0]), Eo) <= 1e-12
    assert _frel(eng.unpack(F, 0), Fo) <= 1e-12


def test_pair_large_periodic_sampled():
    """N = 4096, P = 64 in its periodic box: the energy against the whole
    double sum, forces at sampled beads one by one."""
    s = inputs.config_large()
    eng, pos = _engine([s], box=s.box, pair=(G, SIG))
    F, E = eng.pair_forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    Eo, _ = pair_gaussian(s.R, G, SIG, L=s.box, forces=False, rows=512)
    assert _rel(float(E[0]), Eo) <= 1e-12
    Fg = eng.unpack(F, 0)
    rng = np.random.default_rng(11)
    ref = []
    got = []
    for a, j in zip(rng.integers(0, s.N, 40), rng.integers(0, s.P, 40)):
        ref.append(pair_gaussian_at(s.R, G, SIG, s.box, a, j))
        got.append(Fg[a, j])
    ref, got = np.array(ref), np.array(got)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_pair_added_to_exchange_everywhere():
    """A batch of uneven systems with the trap and the pair interaction:
    forces, energy-only, the batched entry and the distinguishable path
    each equal their pair-free result plus the pair oracle's; the original
    algorithm agrees too."""
    systems = [System(cube_system(n, p, seed=n), beta=b) for n, p, b in [(40, 4, 1.0), (129, 8, 0.7), (300, 6, 1.3)]]
    trap = 0.6
    eng, pos = _engine(systems, trap=trap, pair=(G, SIG))
    ref, _ = _engine(systems, trap=trap)
    orig, _ = _engine(systems, trap=trap, pair=(G, SIG), algorithm="original")
    F, E = eng.forces(pos)
    E_only = eng.energy(pos)
    Fb = eng.empty()
    Eb = torch.empty(len(systems), dtype=torch.float64, device=pos.device)
    offs = torch.tensor(eng.offsets, dtype=torch.int64, device=pos.device)
    eng.forces_batched(pos, offs, Fb, Eb)
    Fd, Ed = eng.distinguishable(pos)
    F0, E0 = ref.forces(pos)
    Fd0, Ed0 = ref.distinguishable(pos)
    Fo, Eo = orig.forces(pos)
    torch.cuda.synchronize()
    for e in (eng, ref, orig):
        assert e.status() == 0
    assert torch.equal(E_only, E) and torch.equal(Eb, E) and torch.equal(Fb, F)
    # a negative caller offset skips its system in the pair launch as well
    offs2 = offs.clone()
    offs2[1] = -1
    Fb.fill_(5.0)
    Eb.fill_(123.0)
    eng.forces_batched(pos, offs2, Fb, Eb)
    torch.cuda.synchronize()
    assert eng.status() == 4  # PIMDB_STATUS_RANGE
    assert float(Eb[1]) == 123.0 and float(Eb[0]) == float(E[0]) and float(Eb[2]) == float(E[2])
    o1 = eng.offsets[1]
    assert bool((Fb[o1:o1 + 3 * systems[1].P * systems[1].N] == 5.0).all())
    for i, s in enumerate(systems):
        Ep, Fp = pair_gaussian(s.R, G, SIG)
        for (Fx, Ex, Fy, Ey) in [(F, E, F0, E0), (Fd, Ed, Fd0, Ed0), (Fo, Eo, F0, E0)]:
            assert _rel(float(Ex[i]), float(Ey[i]) + Ep) <= TOL
            assert _frel(eng.unpack(Fx, i), ref.unpack(Fy, i) + Fp) <= TOL
    # and the total against the long-double exchange oracle plus trap and pair
    for i, s in enumerate(systems):
        o = oracle.alg1(s.R, s.beta, s.m, s.omegaP, precision="f80", extras=False)
        c = s.m * trap * trap / s.P
        Ep, Fp = pair_gaussian(s.R, G, SIG)
        assert _rel(float(E[i]), o["V"] + 0.5 * c * float((s.R ** 2).sum()) + Ep) <= TOL
        assert _frel(eng.unpack(F, i), o["F"] - c * s.R + Fp) <= TOL


def test_pair_in_autograd_and_static():
    """The autograd forward half includes U-bar and its backward half the
    pair gradient; the static-scratch entry matches the workspace entry."""
    s = System(gaussian_system(200, 8, seed=4), beta=1.0)
    eng, pos = _engine([s], pair=(G, SIG))
    F, E = eng.forces(pos)
    p = pos.clone().requires_grad_(True)
    V = exchange_potential(p, eng)
    (2.5 * V.sum()).backward()
    Fs, Es = eng.forces_static(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    assert _rel(float(V.detach()[0]), float(E[0])) <= 1e-14
    assert float((p.grad + 2.5 * F).abs().max()) <= 1e-12 * float(F.abs().max())
    assert torch.equal(Fs, F) and torch.equal(Es, E)


def test_pair_md_step_matches_host():
    """One velocity-Verlet step with the pair interaction: the device step
    equals the same kick-drift-kick on the host with the oracle forces."""
    s = System(cube_system(64, 4, seed=8), beta=1.0)
    eng, pos = _engine([s], pair=(G, SIG))
    vel = eng.pack(inputs.initial_velocities(s.N, s.P, s.beta, s.m, seed=3))
    F = eng.empty()
    E = torch.empty(1, dtype=torch.float64, device=pos.device)
    eng.forces(pos, out=F, energy=E)
    R0 = eng.unpack(pos, 0)
    V0 = eng.unpack(vel, 0)
    dt = 0.01
    eng.md_step(pos, vel, F, E, dt)
    torch.cuda.synchronize()
    assert eng.status() == 0

    def force(R):
        o = oracle.alg1(R, s.beta, s.m, s.omegaP, precision="f80", extras=False)
        return o["F"] + pair_gaussian(R, G, SIG)[1]

    f0 = force(R0)
    v_half = V0 + 0.5 * dt * f0 / s.m
    R1 = R0 + dt * v_half
    V1 = v_half + 0.5 * dt * force(R1) / s.m
    assert np.abs(eng.unpack(pos, 0) - R1).max() <= 1e-12 * np.abs(R1).max()
    assert np.abs(eng.unpack(vel, 0) - V1).max() <= 1e-10 * np.abs(V1).max()


def test_pair_arguments():
    s = System(cube_system(20, 4, seed=1), beta=1.0)
    eng, pos = _engine([s])
    lib, h = eng.lib, eng._h
    assert lib.pimdb_set_pair_gaussian(h, float("nan"), 1.0) == _lib.PIMDB_EINVAL
    assert lib.pimdb_set_pair_gaussian(h, 1.0, 0.0) == _lib.PIMDB_EINVAL
    assert lib.pimdb_set_pair_gaussian(h, 1.0, float("inf")) == _lib.PIMDB_EINVAL
    F = eng.empty()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    assert lib.pimdb_pair_forces(h, p(pos), p(F), None) == _lib.PIMDB_EINVAL  # none set
    eng.set_pair_gaussian(G, SIG)
    Fp, Ep = eng.pair_forces(pos)
    eng.set_pair_gaussian(0.0)
    F0, E0 = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    ref = BosonicExchange(s.N, s.P, s.beta)
    F1, E1 = ref.forces(ref.pack(s.R))
    torch.cuda.synchronize()
    assert torch.equal(F0, F1) and torch.equal(E0, E1)
    assert float(Ep[0]) > 0.0
