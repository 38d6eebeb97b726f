"""GPU: split recursions (each system's forward and backward recursion
spread over a chain workgroup and helper workgroups on other CUs) against
the whole recursions and the long-double oracle, in every entry point, in
graph replays, and the bounded waits' failure path."""
import concurrent.futures as cf
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2305_18025_amd import BosonicExchange, VelocityVerlet, exchange_potential, inputs
from paper_2305_18025_amd.inputs import System, cube_system, gaussian_system

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOLMIX = 1e-5
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _engine(systems, **kw):
    eng = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems], **kw)
    return eng, eng.pack([s.R for s in systems])


def _oracle_f80(s):
    return oracle.alg1(s.R, s.beta, s.m, s.omegaP, L=s.box, precision="f80", extras=False)


def _assert_parity(eng, F, E, systems, tol):
    with cf.ThreadPoolExecutor(min(8, len(systems))) as ex:
        refs = list(ex.map(_oracle_f80, systems))
    for i, (s, o) in enumerate(zip(systems, refs)):
        ee = abs(float(E[i]) - o["V"]) / abs(o["V"])
        fe = float(np.abs(eng.unpack(F, i) - o["F"]).max() / np.abs(o["F"]).max())
        print("  %s: energy %.2e forces %.2e" % (s.name or "N%d" % s.N, ee, fe))
        assert ee <= tol and fe <= tol, (i, ee, fe)


@pytest.mark.parametrize("g", [1, 3, 7, 14])
def test_split_equals_whole(g):
    """Systems of 129 (one helper block), 300, 1024 and 2049 particles (a
    ragged last block) in one batch: the split launch with g blocks per
    helper agrees with the whole recursions to rounding."""
    systems = [System(cube_system(n, 8, seed=n), beta=b, name="N%d" % n)
               for n, b in [(129, 1.0), (300, 0.7), (1024, 1.0), (2049, 1.3)]]
    sp, pos = _engine(systems, split=g)
    assert sp.split[0] == g and sp.split[1] > 0
    per = sp.tuning[1]
    wh = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                         [s.m for s in systems], [s.omegaP for s in systems], split=0, threads=512, per_thread=8)
    F1, E1 = sp.forces(pos)
    F0, E0 = wh.forces(pos)
    torch.cuda.synchronize()
    assert sp.status() == 0 and wh.status() == 0
    print("g=%d: %d helpers, %d rows per thread" % (g, sp.split[1], per))
    if g == 7:
        _assert_parity(sp, F1, E1, systems, TOL64)
    # the whole-recursion reference at 512 threads with 8 rows: the same
    # terms, summed in slightly different slices (the split chain shares
    # the previous block's terms among all its waves)
    assert ((E1 - E0).abs() <= 1e-14 * E0.abs()).all()
    assert (F1 - F0).abs().max() <= 1e-13 * F0.abs().max()


def test_split_plain_headline_automatic():
    """One N=1024, P=32 system: the library splits it by itself."""
    s = inputs.config_headline()
    eng, pos = _engine([s])
    assert eng.split[0] > 0
    F, E = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    _assert_parity(eng, F, E, [s], TOL64)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_split_large_periodic(precision):
    """The periodic N=4096, P=64 system with split recursions."""
    s = inputs.config_large()
    eng, pos = _engine([s], box=s.box, precision=precision)
    assert eng.split[0] > 0
    F, E = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    _assert_parity(eng, F, E, [s], TOL64 if precision == "fp64" else TOLMIX)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_split_shared_cu_periodic(precision):
    """Periodic systems whose split plan puts two workgroups on a CU (the
    8-wave chain with lag 2, whose slot waves form the next block's terms
    from the published step values while the steps run), in the direct
    forms (FP64 and mixed): against the long-double oracle and against the
    whole recursions to rounding."""
    L = 6.0
    systems = [System(cube_system(n, 8, seed=n, side=L), beta=b, box=L, name="N%d" % n)
               for n, b in [(300, 1.0), (577, 0.8), (1024, 1.2), (1500, 0.9)] * 4]
    sp, pos = _engine(systems, box=L, precision=precision, split=1)
    assert sp.split[0] == 1 and sp.split[1] > 0 and sp.split[2] == 0  # two workgroups per CU
    wh = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                         [s.m for s in systems], [s.omegaP for s in systems], box=L, precision=precision,
                         split=0, threads=512, per_thread=8)
    F1, E1 = sp.forces(pos)
    F0, E0 = wh.forces(pos)
    torch.cuda.synchronize()
    assert sp.status() == 0 and wh.status() == 0
    _assert_parity(sp, F1, E1, systems[:4], TOL64 if precision == "fp64" else TOLMIX)
    assert ((E1 - E0).abs() <= 1e-14 * E0.abs()).all()
    assert (F1 - F0).abs().max() <= 1e-13 * F0.abs().max()


def test_split_open_maximum_size():
    systems = [System(cube_system(4096, 8, seed=21), beta=1.0, name="open N4096"),
               System(cube_system(4033, 8, seed=22), beta=1.5, name="open N4033")]
    eng, pos = _engine(systems, split=7)
    F, E = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    _assert_parity(eng, F, E, systems, TOL64)


def test_split_energy_and_adjoint():
    """Energy-only calls (forward recursion alone) and the autograd adjoint
    (backward recursion alone) on split recursions."""
    systems = [System(gaussian_system(700, 16, seed=7), beta=1.0, name="N700"),
               System(cube_system(1500, 8, seed=8), beta=0.6, name="N1500")]
    eng, pos = _engine(systems, split=7)
    E = eng.energy(pos)
    p = pos.clone().requires_grad_(True)
    V = exchange_potential(p, eng)
    V.sum().backward()
    F, E2 = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    assert torch.equal(E, E2) and torch.equal(V.detach(), E2)
    assert torch.equal(p.grad, -F)
    _assert_parity(eng, F, E2, systems, TOL64)


def test_split_graph_replays_and_md():
    """A graph of split-recursion MD steps replays exactly like eager steps,
    with eager calls between the replays (the flags must be clear at the
    start of every evaluation)."""
    systems = [System(cube_system(n, pp, seed=n + pp), beta=b) for n, pp, b in [(900, 8, 1.0), (300, 16, 0.6)]]
    eng, pos = _engine(systems, trap=1.0, split=7)
    vel = eng.pack([inputs.initial_velocities(s.N, s.P, s.beta, s.m, seed=1) for s in systems])
    a = VelocityVerlet(eng, pos.clone(), vel.clone(), 0.01)
    b = VelocityVerlet(eng, pos.clone(), vel.clone(), 0.01)
    b.capture(steps_per_replay=3)
    for _ in range(3):
        a.step(3)
        b.replay(1)
        torch.cuda.synchronize()
        _ = eng.energy(a.pos)
        torch.cuda.synchronize()
        assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel) and torch.equal(a.forces, b.forces)
    assert eng.status() == 0


def test_split_static_scratch_entry():
    """The entry point without a workspace on split recursions, after a
    whole-recursion call left other contents in the static scratch."""
    s = inputs.config_headline()
    whole, pos = _engine([s], split=0)
    whole.forces_static(pos)
    torch.cuda.synchronize()
    eng = BosonicExchange(s.N, s.P, s.beta, s.m, s.omegaP, split=7)
    F0, E0 = eng.forces(pos)
    F1, E1 = eng.forces_static(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    assert torch.equal(F0, F1) and torch.equal(E0, E1)


def test_split_wait_timeout_reports_and_exits():
    """With the split waits' time limit set to zero (from the environment,
    read when the handle is created) every wait gives up at once: each
    workgroup exits normally, the call returns, and the status word reports
    PIMDB_STATUS_TIMEOUT.  Run in a child process so the setting stays
    there."""
    code = r"""
import os, sys, torch
sys.path.insert(0, %r)
from paper_2305_18025_amd import BosonicExchange, inputs
s = inputs.config_headline()
eng = BosonicExchange(s.N, s.P, s.beta, s.m, s.omegaP, split=7)
pos = eng.pack(s.R)
eng.forces(pos)
torch.cuda.synchronize()
st = eng.status()
print("status", st, flush=True)
assert st & 16, st
""" % ROOT
    env = dict(os.environ, PIMDB_SPLIT_WAIT_US="0")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0
