"""Scaled pair interaction U-bar and the closing-spring table -- CPU oracle
(test infrastructure only: tests, the smoke check and the bench's CPU
baseline use it; the library never does).

The paper's partition function weights every imaginary-time slice with the
interaction scaled by 1/P (Theory, the bosonic partition function):

    U-bar = (1/P) sum_{j=1}^{P} sum_{a<b} U(|r_a^j - r_b^j|),

and its interacting benchmarks use pair potentials (Methods, "Simulation
details").  Here U is a caller-parameterised Gaussian,

    U(r) = g exp(-r^2 / (2 sigma^2)),

whose force on bead j of particle a is

    F_a^j = -dU-bar/dr_a^j = (1/P) sum_{b != a} (g / sigma^2) exp(-r_ab^2 / (2 sigma^2)) (r_a^j - r_b^j).

g and sigma are inputs; no parameter of the paper's systems is assumed.
Periodic boxes (L > 0) take the minimum image d - L rint(d / L) (half to
even), as the springs do.  Positions are (N, P, 3), FP64.
"""
from __future__ import annotations

import numpy as np


def _image(d, L):
    return d - L * np.rint(d / L) if L > 0 else d


def pair_gaussian(R, g, sigma, L=0.0, forces=True, rows=256):
    """U-bar and its forces (N, P, 3) by the double sum over pairs, one bead
    slice at a time (rows of `rows` particles against all particles)."""
    R = np.asarray(R, dtype=np.float64)
    N, P, _ = R.shape
    inv2s2 = 1.0 / (2.0 * sigma * sigma)
    E = 0.0
    F = np.zeros_like(R) if forces else None
    for j in range(P):
        X = R[:, j, :]
        for a0 in range(0, N, rows):
            a1 = min(N, a0 + rows)
            D = _image(X[a0:a1, None, :] - X[None, :, :], L)  # (rows, N, 3): r_a - r_b
            U = g * np.exp(-(D * D).sum(axis=2) * inv2s2)
            U[np.arange(a1 - a0), np.arange(a0, a1)] = 0.0  # no self pair
            E += 0.5 * U.sum()  # each unordered pair is met twice
            if forces:
                F[a0:a1, j, :] += (U[:, :, None] * D).sum(axis=1) / (sigma * sigma)
    if forces:
        F /= P
    return E / P, F


def pair_gaussian_at(R, g, sigma, L, a, j):
    """Force (3,) on bead j of particle a alone (for sampled checks of
    systems too large for the whole double sum)."""
    R = np.asarray(R, dtype=np.float64)
    N, P, _ = R.shape
    D = _image(R[a, j, :][None, :] - R[:, j, :], L)
    U = g * np.exp(-(D * D).sum(axis=1) / (2.0 * sigma * sigma))
    U[a] = 0.0
    return (U[:, None] * D).sum(axis=0) / (sigma * sigma) / P


def endpoint_springs(R, k, L=0.0):
    """The closing-spring table s(v, u) = k |r_v^P - r_u^1|^2 for u <= v
    (Background: the spring that closes the ring of particles u..v runs from
    bead P of v to bead 1 of u), rows v = 1..N concatenated, each holding
    u = 1..v; minimum image when L > 0."""
    R = np.asarray(R, dtype=np.float64)
    N = R.shape[0]
    rows = []
    for v in range(N):
        d = _image(R[v, -1, None, :] - R[:v + 1, 0, :], L)
        rows.append(k * (d * d).sum(axis=1))
    return np.concatenate(rows)


def pair_brute(R, g, sigma, L=0.0):
    """The same double sum written as plain loops over slices and pairs
    (small systems only)."""
    R = np.asarray(R, dtype=np.float64)
    N, P, _ = R.shape
    E = 0.0
    F = np.zeros_like(R)
    for j in range(P):
        for a in range(N):
            for b in range(a + 1, N):
                d = [R[a, j, c] - R[b, j, c] for c in range(3)]
                if L > 0:
                    d = [x - L * float(np.rint(x / L)) for x in d]
                r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
                u = g * float(np.exp(-r2 / (2.0 * sigma * sigma)))
                E += u / P
                for c in range(3):
                    f = u / (sigma * sigma) * d[c] / P
                    F[a, j, c] += f
                    F[b, j, c] -= f
    return E, F
