"""The forward recurrence expanded into compositions (TEST INFRASTRUCTURE).

Unrolling the recurrence for V^[1,N] (Background, recurrence over the length
k of the cycle that contains N) turns exp(-beta V^[1,N]) into a sum over the
2^(N-1) ways of cutting [1, N] into consecutive blocks [u_1, v_1], ...,
[u_m, v_m] with v_m = N: each block is one cycle, and the weight is the product
over blocks of 1/v_i (the factor 1/v of the recurrence taken at each block's
end).  For N = 3 this is the expansion the paper writes out with weights 1/6,
1/3, 1/6, 1/3.  Each composition is one representative permutation
(appendix "Some Combinatorics of Permutations": 2^(N-1) of them).

Cycle energies here come from their definition (Background, the cycle energy
as a double sum over the particles of the cycle and all P springs, the last
bead of v connected back to the first bead of u), not from the incremental
recurrence.  Feasible for N <= 16.
"""
from __future__ import annotations

import math

import numpy as np


def _mi(d, L):
    if L > 0:
        return d - L * np.round(d / L)
    return d


def cycle_energy(R, u, v, k, L=0.0):
    """E^[u,v] (1-based, u <= v) from the definition."""
    idx = np.arange(u - 1, v)
    ring = R[idx]  # (n, P, 3)
    nxt = np.empty_like(ring)
    nxt[:, :-1, :] = ring[:, 1:, :]
    nxt[:-1, -1, :] = ring[1:, 0, :]
    nxt[-1, -1, :] = ring[0, 0, :]
    d = _mi(ring - nxt, L)
    return k * math.fsum((d * d).ravel())


def compositions(n):
    """All compositions of [1, n] as lists of (u, v) blocks."""
    out = []
    for mask in range(1 << (n - 1)):
        blocks = []
        u = 1
        for cut in range(1, n):
            if mask >> (cut - 1) & 1:
                blocks.append((u, cut))
                u = cut + 1
        blocks.append((u, n))
        out.append(blocks)
    return out


def composition_weight(blocks):
    return math.prod(1.0 / v for _, v in blocks)


def exchange(R, beta, m, omegaP, L=0.0):
    """V^[1,N] and connection probabilities from the composition sum.

    Returns dict(V, Pr) with Pr[l-1, l'-1] = Pr[l -> l'].
    """
    R = np.ascontiguousarray(R, dtype=np.float64)
    N = R.shape[0]
    if N > 16:
        raise ValueError("composition sum limited to N <= 16")
    k = 0.5 * m * omegaP ** 2
    E = {}
    for v in range(1, N + 1):
        for u in range(1, v + 1):
            E[(u, v)] = cycle_energy(R, u, v, k, L)
    comps = compositions(N)
    logw = np.array([math.log(composition_weight(b)) - beta * sum(E[blk] for blk in b) for b in comps])
    mx = logw.max()
    w = np.exp(logw - mx)
    Z = math.fsum(w)
    V = -(mx + math.log(Z)) / beta
    p = w / Z
    Pr = np.zeros((N, N))
    for pi, blocks in zip(p, comps):
        for (u, v) in blocks:
            for l in range(u, v):
                Pr[l - 1, l] += pi  # l -> l+1 inside a cycle
            Pr[v - 1, u - 1] += pi  # cycle closes v -> u
    return dict(V=V, Pr=Pr)
