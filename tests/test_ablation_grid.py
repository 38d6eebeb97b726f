"""CPU: where the simple two-candidate shift of the recurrences fails, over a
grid of system size N, bead count P, inverse temperature beta and geometry
(appendix "Numerical Stability": any shift is exact in exact arithmetic; the
smallest-exponent shift keeps every shifted exponential at most 1, the
two-candidate shift only the two candidates).

With the two-candidate shift every sum still holds a term equal to one, so
nothing underflows; it fails only when some term's exponent lies more than
ln(DBL_MAX) = 709.78 above the shift's (the exponential overflows).  The
gap is computed here from the long-double oracle's potentials and cycle
energies, for the forward and the backward recursion, and each case is
pinned to the outcome it predicts: the FP64 two-candidate recursion is
exact (energy 1e-12, forces 1e-10 plus the FP64 recursions' own rounding
bound, against the long-double oracle) below the threshold and non-finite
above it; the smallest-exponent shift is exact everywhere.  Run as a
script, this file prints the table of the outcomes.
"""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2305_18025_amd.inputs import cube_system, gaussian_system, omega_p  # noqa: E402

LN_MAX = math.log(np.finfo(np.float64).max)  # 709.78
BAND = 8.0  # gaps within this of the threshold are not pinned either way

GEOMETRIES = ("gaussian", "cube", "pairs", "chain")


def geometry(name, N, P, seed):
    """Positions (N, P, 3) of the four geometries of the grid:
    gaussian  cold cluster, centroids N(0, 1), beads jittered 0.3;
    cube      liquid-like, centroids uniform at unit mean spacing;
    pairs     linked pairs, ring 2i ends where ring 2i+1 starts (strong
              two-particle exchange, the pair about 2 k c^2 below the
              separate rings), c = 6, pairs 30 apart;
    chain     particles in label order 2 apart on a line (long rings
              favoured across neighbours only)."""
    if name == "gaussian":
        return gaussian_system(N, P, seed)
    if name == "cube":
        return cube_system(N, P, seed)
    rng = np.random.default_rng(seed)
    if name == "pairs":
        c, D = 6.0, 30.0
        R = np.zeros((N, P, 3))
        f = np.linspace(0.0, 1.0, P)[:, None]
        for i in range(N // 2):
            A = np.array([D * i, 0.0, 0.0])
            B = A + np.array([0.0, c, 0.0])
            R[2 * i] = A + (B - A) * f
            R[2 * i + 1] = B + (A - B) * f
        if N % 2:
            R[N - 1] = np.array([D * (N // 2), 0.0, 0.0])
        return R + rng.normal(0.0, 0.05, R.shape)
    if name == "chain":
        c = np.zeros((N, 3))
        c[:, 0] = 2.0 * np.arange(N)
        return c[:, None, :] + rng.normal(0.0, 0.3, (N, P, 3))
    raise ValueError(name)


def shift_gaps(o, beta):
    """Largest beta (shift - smallest exponent) over the steps of the forward
    and the backward recursion under the two-candidate shift, from the
    oracle's V^[1,v], V^[u,N] and E^[u,v]."""
    E, Vf, Vb = o["E"], o["Vf"], o["Vb"]
    N = E.shape[0]
    gf = gb = 0.0
    for v in range(1, N + 1):
        x = Vf[:v] + E[:v, v - 1]  # u = 1..v: V^[1,u-1] + E^[u,v]
        gf = max(gf, beta * (min(x[0], x[v - 1]) - x.min()))
    for u in range(N, 0, -1):
        y = E[u - 1, u - 1:] + Vb[u + 1:N + 2]  # l = u..N: E^[u,l] + V^[l+1,N]
        gb = max(gb, beta * (min(y[0], y[-1]) - y.min()))
    return gf, gb


def case(oracle, geo, N, P, beta, seed=7):
    R = geometry(geo, N, P, seed)
    w = omega_p(P, beta)
    ref = oracle.alg1(R, beta, 1.0, w, precision="f80", extras=True)
    gf, gb = shift_gaps(ref, beta)
    two = oracle.alg1(R, beta, 1.0, w, precision="f64", shift_mode=1, extras=False)
    mn = oracle.alg1(R, beta, 1.0, w, precision="f64", shift_mode=0, extras=False)
    rel = lambda a, b: abs(a - b) / abs(b)
    frel = lambda F, G: float(np.abs(F - G).max() / np.abs(G).max())
    # the FP64 recursions' own rounding: exponents of size beta |V| lose
    # about beta |V| 2^-53 absolutely; a probability that small absolute
    # error leaves times its spring's pull (m w^2 times the link length, at
    # most the longest link) reaches the forces
    link = float(np.linalg.norm(R[1:, 0] - R[:-1, -1], axis=1).max()) if N > 1 else 0.0
    amp = max(1.0, w * w * link / float(np.abs(ref["F"]).max()))
    out = {"gap": max(gf, gb), "gap_fwd": gf, "gap_bwd": gb,
           "ftol": 1e-10 + 16.0 * beta * abs(ref["V"]) * 2.0 ** -53 * amp,
           "min_V": rel(mn["V"], ref["V"]), "min_F": frel(mn["F"], ref["F"])}
    finite = math.isfinite(two["V"]) and bool(np.isfinite(two["F"]).all())
    out["two_finite"] = finite
    if finite:
        out["two_V"] = rel(two["V"], ref["V"])
        out["two_F"] = frel(two["F"], ref["F"])
    return out


GRID = [(g, N, P, b) for g in GEOMETRIES for N in (8, 32, 96) for P in (4, 16, 64) for b in (0.5, 2.0, 8.0)]
# the headline's size, cold and hot
GRID += [(g, 1024, 32, b) for g in ("gaussian", "cube") for b in (0.25, 1.0)]


@pytest.mark.parametrize("geo,N,P,beta", GRID)
def test_two_candidate_shift_boundary(oracle_lib, geo, N, P, beta):
    r = case(oracle_lib, geo, N, P, beta)
    assert r["min_V"] < 1e-12 and r["min_F"] < r["ftol"], r
    if r["gap"] < LN_MAX - BAND:
        assert r["two_finite"], r
        assert r["two_V"] < 1e-12 and r["two_F"] < r["ftol"], r
    elif r["gap"] > LN_MAX + BAND:
        assert not r["two_finite"], r


def test_grid_has_both_outcomes(oracle_lib):
    """The grid reaches both sides of the threshold, so the pins above test
    the boundary and not just one regime."""
    gaps = [case(oracle_lib, g, N, P, b)["gap"] for g, N, P, b in
            [("pairs", 32, 64, 0.5), ("gaussian", 8, 4, 2.0)]]
    assert gaps[0] > LN_MAX + BAND and gaps[1] < LN_MAX - BAND, gaps


def table(oracle):
    """Markdown table: per geometry, P and beta, the outcome of the two-
    candidate shift at each N (ok / overflow) with the largest gap."""
    lines = ["| geometry | P | beta | " + " | ".join("N=%d" % n for n in (8, 32, 96)) + " |",
             "|---|---|---|" + "---|" * 3]
    for g in GEOMETRIES:
        for P in (4, 16, 64):
            for b in (0.5, 2.0, 8.0):
                cells = []
                for N in (8, 32, 96):
                    r = case(oracle, g, N, P, b)
                    cells.append("%s (%.0f)" % ("ok" if r["two_finite"] else "overflow", r["gap"]))
                lines.append("| %s | %d | %g | %s |" % (g, P, b, " | ".join(cells)))
    return "\n".join(lines)


if __name__ == "__main__":
    import oracle as _oracle
    _oracle.build(force=False)
    print(table(_oracle))
