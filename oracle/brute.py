"""Brute force over all N! permutations (TEST INFRASTRUCTURE, N <= 8).

Implements, literally:
  * canonical cycle notation (appendix "Cycle Notation of Permutations"):
    start from the smallest element not yet used and follow sigma;
  * the representative permutation G[sigma] (Methods, "Definition of
    G[sigma]"; appendix definition of the representative permutation): sort
    the cycles by their largest element, ascending, then relabel the elements
    1..N consecutively keeping cycle lengths and order;
  * the ring-polymer energy of a permutation E^sigma (Background, the spring
    energy with r_l^{P+1} = r_{sigma(l)}^1);
  * V^[1,N] as the average over all sigma of exp(-beta E^{G[sigma]})
    (Theory, "Potential as a sum over representative permutations");
  * the force as the expectation of -grad E^{G[sigma]} under the Boltzmann
    distribution of representative permutations, and the connection
    probabilities Pr[l -> l'] as the total probability of the permutations
    whose representative maps l to l' (Theory, "Force as an expectation
    value", "Force on exterior beads");
  * V_sym, the symmetric potential over all permutations without G
    (Background), which the paper notes differs from V^[1,N].

Permutations are 1-based tuples: ``sigma[l-1] = sigma(l)``.
Positions use the oracle layout R[l, j, c] of shape (N, P, 3).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def cycles(sigma):
    """Canonical cycle notation: list of cycles (tuples), each starting at the
    smallest element not yet placed, following l -> sigma(l)."""
    n = len(sigma)
    seen = [False] * (n + 1)
    out = []
    for start in range(1, n + 1):
        if seen[start]:
            continue
        cyc = []
        l = start
        while not seen[l]:
            seen[l] = True
            cyc.append(l)
            l = sigma[l - 1]
        out.append(tuple(cyc))
    return out


def from_cycles(cyc_list, n):
    """Permutation (1-based tuple) from a list of cycles."""
    sigma = [0] * n
    for cyc in cyc_list:
        for i, l in enumerate(cyc):
            sigma[l - 1] = cyc[(i + 1) % len(cyc)]
    return tuple(sigma)


def representative(sigma):
    """G[sigma]: cycles sorted by their largest element, then the elements
    replaced by 1..N consecutively, keeping lengths and order."""
    cyc = sorted(cycles(sigma), key=max)
    new = []
    start = 0
    for c in cyc:
        new.append(tuple(range(start + 1, start + len(c) + 1)))
        start += len(c)
    return from_cycles(new, len(sigma))


def _mi(d, L):
    if L > 0:
        return d - L * np.round(d / L)  # numpy rounds half to even
    return d


def perm_energy(R, sigma, k, L=0.0):
    """E^sigma = k sum_l sum_{j=1..P} |r_l^j - r_l^{j+1}|^2 with
    r_l^{P+1} = r_{sigma(l)}^1 (minimum image per spring when L > 0)."""
    N, P, _ = R.shape
    nxt = np.empty_like(R)
    nxt[:, :-1, :] = R[:, 1:, :]
    nxt[:, -1, :] = R[np.asarray(sigma) - 1, 0, :]
    d = _mi(R - nxt, L)
    return k * math.fsum((d * d).ravel())


def perm_forces(R, sigma, k, L=0.0):
    """-grad E^sigma: each bead pulled by its two ring neighbours,
    -m w_P^2 ((r - r_prev) + (r - r_next)) with m w_P^2 = 2k."""
    N, P, _ = R.shape
    inv = np.empty(N, dtype=int)
    inv[np.asarray(sigma) - 1] = np.arange(N)
    prev = np.empty_like(R)
    prev[:, 1:, :] = R[:, :-1, :]
    prev[:, 0, :] = R[inv, -1, :]
    nxt = np.empty_like(R)
    nxt[:, :-1, :] = R[:, 1:, :]
    nxt[:, -1, :] = R[np.asarray(sigma) - 1, 0, :]
    return -2.0 * k * (_mi(R - prev, L) + _mi(R - nxt, L))


def _logmeanexp(x):
    x = np.asarray(x, dtype=np.float64)
    mx = x.max()
    return mx + math.log(math.fsum(np.exp(x - mx)) / len(x))


def exchange(R, beta, m, omegaP, L=0.0, with_forces=True):
    """Brute-force V^[1,N], forces and Pr over all N! permutations.

    Returns dict(V, F, Pr, Vsym, counts) where ``counts`` maps each
    representative permutation to the number of sigma with that G[sigma].
    """
    R = np.ascontiguousarray(R, dtype=np.float64)
    N, P, _ = R.shape
    if N > 9:
        raise ValueError("brute force is limited to N <= 9")
    k = 0.5 * m * omegaP ** 2
    counts = {}
    for sigma in itertools.permutations(range(1, N + 1)):
        g = representative(sigma)
        counts[g] = counts.get(g, 0) + 1
    reps = list(counts)
    e_rep = np.array([perm_energy(R, g, k, L) for g in reps])
    mult = np.array([counts[g] for g in reps], dtype=np.float64)
    # log of (1/N!) sum_sigma exp(-beta E^{G[sigma]}) = log sum_g (mult/N!) exp(-beta E_g)
    logw = -beta * e_rep + np.log(mult) - math.lgamma(N + 1)
    mx = logw.max()
    Z = math.fsum(np.exp(logw - mx))
    V = -(mx + math.log(Z)) / beta
    prob = np.exp(logw - mx) / Z  # Pr(G[sigma]) summed over each class
    Pr = np.zeros((N, N))
    for p, g in zip(prob, reps):
        for l in range(N):
            Pr[l, g[l] - 1] += p
    F = None
    if with_forces:
        F = np.zeros_like(R)
        for p, g in zip(prob, reps):
            F += p * perm_forces(R, g, k, L)
    # symmetric potential over all permutations, no representative map
    e_all = [perm_energy(R, s, k, L) for s in itertools.permutations(range(1, N + 1))]
    Vsym = -_logmeanexp(-beta * np.asarray(e_all)) / beta
    return dict(V=V, F=F, Pr=Pr, Vsym=Vsym, counts=counts)
