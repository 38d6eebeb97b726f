"""CPU pins of the pair-interaction oracle (oracle/pair.py): the two-particle
closed form, plain loops, translation invariance and Newton's third law,
finite differences of the energy, the minimum image, and the sampled form."""
import math

import numpy as np
import pytest

import oracle
from oracle.pair import endpoint_springs, pair_brute, pair_gaussian, pair_gaussian_at
from paper_2305_18025_amd.inputs import cube_system, gaussian_system


def test_two_particles_closed_form():
    """N = 2: U-bar = (1/P) sum_j g exp(-|d_j|^2 / (2 s^2)), and the force on
    particle 1 is minus the derivative of that with respect to r_1^j:
    (g / (P s^2)) exp(-|d_j|^2 / (2 s^2)) d_j, particle 2 the opposite."""
    g, s, P = 2.5, 0.7, 4
    rng = np.random.default_rng(1)
    R = rng.normal(0.0, 0.6, (2, P, 3))
    E, F = pair_gaussian(R, g, s)
    e_ref = 0.0
    for j in range(P):
        d = R[0, j] - R[1, j]
        r = math.sqrt(float(d @ d))
        e_ref += g * math.exp(-r * r / (2 * s * s)) / P
        # dU/dr = -(r / s^2) U: the force along d is -(dU/dr) / P
        f = (r / (s * s)) * g * math.exp(-r * r / (2 * s * s)) / P * d / r
        assert np.allclose(F[0, j], f, rtol=1e-14, atol=0)
        assert np.allclose(F[1, j], -f, rtol=1e-14, atol=0)
    assert abs(E - e_ref) <= 1e-15 * abs(e_ref)


@pytest.mark.parametrize("L", [0.0, 2.0])
def test_matches_plain_loops(L):
    R = cube_system(7, 3, seed=4, side=2.0 if L else None)
    E1, F1 = pair_gaussian(R, 3.0, 0.5, L=L, rows=3)
    E2, F2 = pair_brute(R, 3.0, 0.5, L=L)
    assert abs(E1 - E2) <= 1e-14 * abs(E2)
    assert np.abs(F1 - F2).max() <= 1e-14 * np.abs(F2).max()


def test_translation_invariance_and_newton():
    R = gaussian_system(40, 5, seed=2)
    E, F = pair_gaussian(R, 3.0, 0.5)
    E2, F2 = pair_gaussian(R + np.array([3.1, -7.2, 0.4]), 3.0, 0.5)
    assert abs(E2 - E) <= 1e-13 * abs(E)
    assert np.abs(F2 - F).max() <= 1e-12 * np.abs(F).max()
    # internal forces: each slice's forces sum to zero
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).max()


def test_finite_differences():
    R = gaussian_system(12, 3, seed=3)
    g, s = 3.0, 0.5
    _, F = pair_gaussian(R, g, s)
    rng = np.random.default_rng(5)
    h = 1e-5
    for _ in range(12):
        a, j, c = rng.integers(12), rng.integers(3), rng.integers(3)
        Rp, Rm = R.copy(), R.copy()
        Rp[a, j, c] += h
        Rm[a, j, c] -= h
        dE = (pair_gaussian(Rp, g, s, forces=False)[0] - pair_gaussian(Rm, g, s, forces=False)[0]) / (2 * h)
        assert abs(-dE - F[a, j, c]) <= 1e-7 * np.abs(F).max(), (a, j, c)


def test_minimum_image():
    """Two particles L - delta apart along x in a box of side L interact as
    if delta apart; the force points the short way round."""
    L, delta, P = 5.0, 0.3, 2
    R = np.zeros((2, P, 3))
    R[1, :, 0] = L - delta
    E, F = pair_gaussian(R, 1.0, 0.4, L=L)
    R2 = np.zeros((2, P, 3))
    R2[1, :, 0] = -delta
    E2, F2 = pair_gaussian(R2, 1.0, 0.4)
    assert abs(E - E2) <= 1e-15 * E2
    assert np.abs(F - F2).max() <= 1e-15 * np.abs(F2).max()
    assert F[0, 0, 0] > 0.0  # pushed away from the image at -delta, towards +x


def test_sampled_equals_full():
    R = cube_system(50, 4, seed=9, side=3.0)
    _, F = pair_gaussian(R, 2.0, 0.6, L=3.0)
    for a, j in [(0, 0), (17, 3), (49, 1)]:
        assert np.abs(pair_gaussian_at(R, 2.0, 0.6, 3.0, a, j) - F[a, j]).max() <= 1e-14 * np.abs(F).max()


@pytest.mark.parametrize("L", [0.0, 3.0])
def test_endpoint_springs_against_cycle_energies(L):
    """The closing-spring table against the C oracle's cycle energies E^[u,v]
    and interior energies: a one-particle ring is its interior springs plus
    its own closing spring, s(v,v) = E^[v,v] - E_int(v); and for u < v - 1
    the links cancel in E^[u,v] - E^[u,v-1] - E^[v-1,v] + E_int(v-1)
    = s(v,u) - s(v-1,u) - s(v,v-1)."""
    R = cube_system(9, 4, seed=6, side=L if L else None)
    beta = 1.0
    w = 2.0
    o = oracle.alg1(R, beta, 1.0, w, L=L, extras=True)
    k = 0.5 * w * w
    flat = endpoint_springs(R, k, L)
    N = R.shape[0]
    S = np.zeros((N, N))
    pos = 0
    for v in range(N):
        S[v, :v + 1] = flat[pos:pos + v + 1]
        pos += v + 1
    E, Ei = o["E"], o["Eint"]  # E[u-1, v-1] = E^[u,v]
    scale = np.abs(E).max()
    for v in range(N):
        assert abs(S[v, v] - (E[v, v] - Ei[v])) <= 1e-13 * scale
    for v in range(2, N):
        for u in range(v - 1):
            lhs = E[u, v] - E[u, v - 1] - E[v - 1, v] + Ei[v - 1]
            assert abs(lhs - (S[v, u] - S[v - 1, u] - S[v, v - 1])) <= 1e-12 * scale, (u, v)
