"""CPU oracle for the bosonic PIMD exchange potential V^[1,N] and its forces.

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it; the GPU library never imports this.

Contents
--------
* ``pimdb_oracle.c`` / ``oracle_body.h`` -- plain C implementation of the
  quadratic-scaling potential and forces from the main text's defining
  equations (cycle energies, forward and backward recurrences, connection
  probabilities, interior and exterior bead forces), of the original cubic
  algorithm (appendix "Algorithm Pseudocode", Alg. 2) and of the
  definitional backward potentials (appendix "Connection Probabilities"),
  each in IEEE double (``_f64``) and x87 long double (``_f80``).
* ``brute``        -- brute force over all N! permutations with the
  representative map G (Methods, "Definition of G[sigma]").
* ``compositions`` -- the recurrence expanded into the 2^(N-1) compositions
  of [1, N] (the sum over representative permutations grouped by G).
* ``autodiff``     -- the forward recurrence written with torch CPU float64
  ops and differentiated by autograd (an independent force check).

Layout: positions are ``R[l, j, c]`` (particle, bead, component), a float64
array of shape (N, P, 3); forces are returned in the same layout.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "pimdb_oracle.c"), os.path.join(_HERE, "oracle_body.h")]

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle in place (gcc, -O2, no fast-math)."""
    if not force and os.path.exists(_SO):
        newest = max(os.path.getmtime(p) for p in _SRC)
        if os.path.getmtime(_SO) >= newest:
            return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fno-fast-math", "-std=c11", "-Wall", "-shared", "-fPIC",
           "-o", tmp, _SRC[0], "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        for sfx in ("_f64", "_f80"):
            f = getattr(lib, "orc_alg1" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp]
            f = getattr(lib, "orc_alg2" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, ctypes.c_double, dp, dp]
            f = getattr(lib, "orc_backward_def" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, ctypes.c_double, dp]
        lib.orc_long_double_mant_dig.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_R(R):
    R = np.ascontiguousarray(R, dtype=np.float64)
    if R.ndim != 3 or R.shape[2] != 3:
        raise ValueError("R must have shape (N, P, 3)")
    return R


def long_double_mant_dig() -> int:
    return int(_load().orc_long_double_mant_dig())


def alg1(R, beta, m, omegaP, L=0.0, precision="f64", shift_mode=0, forces=True,
         extras=True):
    """Quadratic-scaling potential and forces ("Fast PIMD-B"): V^[1,N],
    forces and intermediates, from the main text's defining equations.

    Returns a dict with ``V`` (float), ``F`` (N,P,3) or None, and when
    ``extras``: ``Vf`` (N+1: V^[1,v]), ``Vb`` (N+2: V^[u,N] at index u),
    ``Pr`` (N,N: Pr[l -> l'] at [l-1, l'-1]), ``E`` (N,N: E^[u,v] at
    [u-1, v-1], upper triangle), ``Eint`` (N).
    """
    R = _check_R(R)
    N, P, _ = R.shape
    lib = _load()
    fn = getattr(lib, "orc_alg1_" + precision)
    V = np.zeros(1)
    F = np.zeros((N, P, 3)) if forces else None
    Vf = np.zeros(N + 1) if extras else None
    Vb = np.zeros(N + 2) if extras else None
    Pr = np.zeros((N, N)) if extras else None
    E = np.zeros((N, N)) if extras else None
    Eint = np.zeros(N) if extras else None
    rc = fn(N, P, _ptr(R), beta, m, omegaP, L, shift_mode, _ptr(V), _ptr(F), _ptr(Vf), _ptr(Vb),
            _ptr(Pr), _ptr(E), _ptr(Eint))
    if rc != 0:
        raise ValueError("oracle alg1 failed with code %d" % rc)
    return dict(V=float(V[0]), F=F, Vf=Vf, Vb=Vb, Pr=Pr, E=E, Eint=Eint)


def alg2(R, beta, m, omegaP, L=0.0, precision="f64", forces=True):
    """Original cubic PIMD-B (Alg. 2): returns (V, F or None)."""
    R = _check_R(R)
    N, P, _ = R.shape
    fn = getattr(_load(), "orc_alg2_" + precision)
    V = np.zeros(1)
    F = np.zeros((N, P, 3)) if forces else None
    rc = fn(N, P, _ptr(R), beta, m, omegaP, L, _ptr(V), _ptr(F))
    if rc != 0:
        raise ValueError("oracle alg2 failed with code %d" % rc)
    return float(V[0]), F


def backward_def(R, beta, m, omegaP, L=0.0, precision="f64"):
    """V^[u,N] (index u = 1..N) from the definitional recursion; O(N^3)."""
    R = _check_R(R)
    N, P, _ = R.shape
    fn = getattr(_load(), "orc_backward_def_" + precision)
    Vb = np.zeros(N + 1)
    rc = fn(N, P, _ptr(R), beta, m, omegaP, L, _ptr(Vb))
    if rc != 0:
        raise ValueError("oracle backward_def failed with code %d" % rc)
    return Vb
