"""GPU: the original cubic algorithm (appendix "Algorithm Pseudocode", the
original method) behind the same ABI, against the CPU oracle's original
algorithm (cycle energies by their definition, the derivative recurrence per
bead) and the long-double quadratic oracle, and against the quadratic GPU
path; its two-candidate shift (appendix "Numerical Stability") on the
device."""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2305_18025_amd import BosonicExchange, _lib
from paper_2305_18025_amd.inputs import System, cube_system, gaussian_system, omega_p

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _engine(systems, **kw):
    eng = BosonicExchange([s.N for s in systems], [s.P for s in systems], [s.beta for s in systems],
                          [s.m for s in systems], [s.omegaP for s in systems], **kw)
    return eng, eng.pack([s.R for s in systems])


def _trap(s, w):
    """Scaled trap potential (1/P) sum (1/2) m w^2 |r|^2 and its force."""
    c = s.m * w * w / s.P
    return 0.5 * c * float((s.R ** 2).sum()), -c * s.R


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _frel(F, ref):
    return float(np.abs(F - ref).max() / np.abs(ref).max())


def _check(eng, F, E, systems, refs, tol, trap=0.0):
    for i, (s, (V, Fr)) in enumerate(zip(systems, refs)):
        et, ft = _trap(s, trap) if trap else (0.0, 0.0)
        ee = _rel(float(E[i]), V + et)
        fe = _frel(eng.unpack(F, i), Fr + ft)
        print("  %s: energy %.2e forces %.2e" % (s.name or "N%d" % s.N, ee, fe), flush=True)
        assert ee <= tol and fe <= tol, (i, ee, fe)


@pytest.mark.parametrize("N,P,box", [(1, 2, 0.0), (2, 3, 0.0), (3, 8, 0.0), (5, 2, 0.0), (8, 8, 2.5),
                                     (17, 4, 0.0), (33, 3, 4.0), (40, 8, 0.0)])
def test_original_matches_oracle_original(N, P, box):
    """Small systems (one and two v-blocks of 32, a workgroup spanning
    several particles, P = 2 where both beads are exterior, periodic boxes)
    against the oracle's original algorithm."""
    R = cube_system(N, P, seed=100 + N, side=box if box else None)
    s = System(R, beta=1.3, box=box, name="N%dP%d" % (N, P))
    eng, pos = _engine([s], box=box, algorithm="original")
    assert eng.algorithm == ("original", "min")
    F, E = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    V2, F2 = oracle.alg2(s.R, s.beta, s.m, s.omegaP, L=box)
    _check(eng, F, E, [s], [(V2, F2)], TOL64)


@pytest.mark.parametrize("N,P", [(100, 8), (257, 32)])
def test_original_matches_long_double_oracle(N, P):
    """Ragged sizes past several v-blocks and workgroups, with a trap, against
    the long-double quadratic oracle (the same potential and forces)."""
    s = System(gaussian_system(N, P, seed=N), beta=1.0, name="N%dP%d" % (N, P))
    eng, pos = _engine([s], trap=0.7, algorithm="original")
    F, E = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    o = oracle.alg1(s.R, s.beta, s.m, s.omegaP, precision="f80", extras=False)
    _check(eng, F, E, [s], [(o["V"], o["F"])], TOL64, trap=0.7)


def _tol_original(s, V):
    """Accuracy of the original formulation in FP64: each weight
    exp(-beta (V^[1,u-1] + E^[u,v] - V^[1,v])) takes a difference of values
    of magnitude up to |V^[1,N]|, so its exponent carries an absolute
    rounding of about beta |V| 2^-53 (a few roundings), which passes to the
    forces as a relative error; 16 roundings of margin on top of 1e-10."""
    return TOL64 + 16.0 * s.beta * abs(V) * 2.0 ** -53


def test_original_equals_fast_at_headline_size():
    """N = 1024, P = 32: the original algorithm on the GPU and the quadratic
    one agree with each other and with the long-double oracle (the original
    one to its rounding bound, about 6e-10 here)."""
    s = System(gaussian_system(1024, 32, seed=3), beta=1.0, name="N1024")
    fast, pos = _engine([s])
    orig, _ = _engine([s], algorithm="original")
    F1, E1 = fast.forces(pos)
    F2, E2 = orig.forces(pos)
    torch.cuda.synchronize()
    assert fast.status() == 0 and orig.status() == 0
    o = oracle.alg1(s.R, s.beta, s.m, s.omegaP, precision="f80", extras=False)
    tol = _tol_original(s, o["V"])
    print("  original-form tolerance %.2e" % tol)
    _check(fast, F1, E1, [s], [(o["V"], o["F"])], TOL64)
    _check(orig, F2, E2, [s], [(o["V"], o["F"])], tol)
    assert _rel(float(E2[0]), float(E1[0])) <= TOL64
    assert _frel(orig.unpack(F2, 0), fast.unpack(F1, 0)) <= tol


def test_original_batch_energy_and_md():
    """A batch of uneven systems, the energy-only entry, and one velocity
    Verlet step equal to the quadratic path's."""
    systems = [System(cube_system(n, p, seed=n), beta=b, name="N%d" % n)
               for n, p, b in [(5, 4, 0.8), (70, 8, 1.0), (129, 6, 1.7)]]
    orig, pos = _engine(systems, trap=0.5, algorithm="original")
    fast, _ = _engine(systems, trap=0.5)
    F, E = orig.forces(pos)
    E_only = orig.energy(pos)
    torch.cuda.synchronize()
    assert orig.status() == 0
    refs = [oracle.alg2(s.R, s.beta, s.m, s.omegaP) for s in systems]
    _check(orig, F, E, systems, refs, TOL64, trap=0.5)
    assert torch.equal(E_only, E)
    vel = torch.zeros_like(pos)
    p1, v1 = pos.clone(), vel.clone()
    p2, v2 = pos.clone(), vel.clone()
    f1, f2 = orig.empty(), fast.empty()
    e1 = torch.empty(len(systems), dtype=torch.float64, device=pos.device)
    e2 = torch.empty_like(e1)
    for eng, p, v, f, e in [(orig, p1, v1, f1, e1), (fast, p2, v2, f2, e2)]:
        eng.forces(p, out=f, energy=e)
        eng.md_step(p, v, f, e, 0.01)
    torch.cuda.synchronize()
    assert orig.status() == 0 and fast.status() == 0
    assert (p1 - p2).abs().max() <= 1e-12 * p2.abs().max()
    assert (v1 - v2).abs().max() <= TOL64 * v2.abs().max()
    assert ((e1 - e2).abs() <= TOL64 * e2.abs()).all()


def _paired(npairs, P, c, D, seed):
    """Linked pairs: the beads of particle 2i run along a segment of length c
    and those of 2i+1 back along it, so each ring's last bead sits on the
    other's first (the pair exchange is favoured by about k c^2)."""
    rng = np.random.default_rng(seed)
    R = np.zeros((2 * npairs, P, 3))
    f = np.linspace(0.0, 1.0, P)[:, None]
    for i in range(npairs):
        A = np.array([D * i, 0.0, 0.0])
        B = A + np.array([0.0, c, 0.0])
        R[2 * i] = A + (B - A) * f
        R[2 * i + 1] = B + (A - B) * f
    return R + rng.normal(0.0, 0.05, R.shape)


@pytest.mark.parametrize("c", [4.0, 8.0, 12.0, 20.0])
def test_two_term_shift_on_device(c):
    """The two-candidate shift on the device: exact (1e-10) where the
    oracle's two-term recurrence is finite, the non-finite status bit where
    its shifted exponentials overflow (beta 2 k c^2 above ln(DBL_MAX)); the
    minimum shift stays exact on every case."""
    P, beta = 8, 1.0
    s = System(_paired(6, P, c, 30.0, seed=1), beta=beta, name="pairs c=%g" % c)
    ref = oracle.alg1(s.R, beta, s.m, s.omegaP, precision="f80", extras=False)
    two_o = oracle.alg1(s.R, beta, s.m, s.omegaP, precision="f64", shift_mode=1, extras=False)
    mn, pos = _engine([s], algorithm="original")
    two, _ = _engine([s], algorithm="original", shift="two_term")
    assert two.algorithm == ("original", "two_term")
    F1, E1 = mn.forces(pos)
    F2, E2 = two.forces(pos)
    torch.cuda.synchronize()
    assert mn.status() == 0
    _check(mn, F1, E1, [s], [(ref["V"], ref["F"])], TOL64)
    st = two.status()
    if math.isfinite(two_o["V"]):
        assert st == 0
        _check(two, F2, E2, [s], [(ref["V"], ref["F"])], TOL64)
    else:
        assert beta * 2 * 4 * c * c > 709.0
        assert st & 2, st  # PIMDB_STATUS_NONFINITE_OUTPUT


def test_original_rejects_other_entries():
    """Entries outside the original path's scope fail with PIMDB_EINVAL;
    the quadratic algorithm takes no shift; switching back works."""
    s = System(cube_system(20, 4, seed=2), beta=1.0)
    eng, pos = _engine([s], algorithm="original")
    lib, h = eng.lib, eng._h
    F = eng.empty()
    E = torch.empty(1, dtype=torch.float64, device=pos.device)
    offs = torch.tensor(eng.offsets, dtype=torch.int64, device=pos.device)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    assert lib.pimdb_exchange_forces_batched(h, p(pos), p(offs), p(F), p(E)) == _lib.PIMDB_EINVAL
    assert lib.pimdb_exchange_forces_static(h, p(pos), p(F), p(E)) == _lib.PIMDB_EINVAL
    assert lib.pimdb_set_algorithm(h, _lib.PIMDB_ALG_FAST, _lib.PIMDB_SHIFT_TWO_TERM) == _lib.PIMDB_EINVAL
    assert lib.pimdb_set_algorithm(h, 7, 0) == _lib.PIMDB_EINVAL
    F0, E0 = eng.forces(pos)
    eng.set_algorithm("fast")
    assert eng.algorithm == ("fast", "min")
    F1, E1 = eng.forces(pos)
    torch.cuda.synchronize()
    assert eng.status() == 0
    assert _rel(float(E1[0]), float(E0[0])) <= TOL64
    assert _frel(eng.unpack(F1, 0), eng.unpack(F0, 0)) <= TOL64
