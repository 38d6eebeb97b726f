"""Seeded synthetic bead configurations.

This module only draws random numbers; it holds none of the method's
arithmetic, so both the GPU path's tests and the CPU oracle can take their
inputs from it.  Units: hbar = m = 1, d = 3; omega_P = sqrt(P) / beta
(the ring-polymer spring frequency of the paper's background section).

Layouts: generators return ``R`` of shape (N, P, 3) (particle, bead,
component).  The GPU library takes bead-major structure-of-arrays
``(P, 3, N)``; :func:`to_soa` / :func:`from_soa` convert.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def omega_p(P: int, beta: float, hbar: float = 1.0) -> float:
    return math.sqrt(P) / (beta * hbar)


def gaussian_system(N: int, P: int, seed, sigma_c: float = 1.0, sigma_b: float = 0.3):
    """Centroids ~ N(0, sigma_c^2) per coordinate; bead = centroid + N(0, sigma_b^2)."""
    rng = np.random.default_rng(seed)
    c = rng.normal(0.0, sigma_c, size=(N, 3))
    return c[:, None, :] + rng.normal(0.0, sigma_b, size=(N, P, 3))


def cube_system(N: int, P: int, seed, side: float | None = None, sigma_b: float = 0.3):
    """Centroids uniform in [0, side)^3 (default side N^(1/3): mean spacing 1);
    bead = centroid + N(0, sigma_b^2)."""
    if side is None:
        side = N ** (1.0 / 3.0)
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, side, size=(N, 3))
    return c[:, None, :] + rng.normal(0.0, sigma_b, size=(N, P, 3))


def to_soa(R) -> np.ndarray:
    """(N, P, 3) -> contiguous (P, 3, N)."""
    return np.ascontiguousarray(np.transpose(np.asarray(R, dtype=np.float64), (1, 2, 0)))


def from_soa(X) -> np.ndarray:
    """(P, 3, N) -> contiguous (N, P, 3)."""
    return np.ascontiguousarray(np.transpose(np.asarray(X, dtype=np.float64), (2, 0, 1)))


@dataclass
class System:
    """One synthetic system: positions (N, P, 3) and its parameters."""
    R: np.ndarray
    beta: float
    m: float = 1.0
    omegaP: float = 0.0
    box: float = 0.0
    name: str = ""

    def __post_init__(self):
        if self.omegaP == 0.0:
            self.omegaP = omega_p(self.R.shape[1], self.beta)

    @property
    def N(self):
        return self.R.shape[0]

    @property
    def P(self):
        return self.R.shape[1]


def config_tiny(seed=1) -> System:
    """N=8, P=8, beta=1, Gaussian centroids N(0,1), bead jitter 0.3."""
    return System(gaussian_system(8, 8, seed), beta=1.0, name="tiny N8 P8 gaussian")


def config_plain(seed=2) -> System:
    """N=256, P=32, beta=1, cube of side 6.35 (mean spacing ~1), jitter 0.3."""
    return System(cube_system(256, 32, seed, side=6.35), beta=1.0, name="plain N256 P32 cube")


def config_headline(seed=3, variant: str = "gaussian") -> System:
    """N=1024, P=32, beta=1.  'gaussian': centroids N(0,1) as in the tiny
    case; 'cube': uniform cube of side 1024^(1/3) (mean spacing 1)."""
    if variant == "gaussian":
        R = gaussian_system(1024, 32, seed)
    elif variant == "cube":
        R = cube_system(1024, 32, seed)
    else:
        raise ValueError(variant)
    return System(R, beta=1.0, name="N1024 P32 " + variant)


def config_batch(seed=4, S: int = 64, n_lo: int = 64, n_hi: int = 2048):
    """S independent systems: N ~ U{n_lo..n_hi}, P ~ {16, 32, 64}, beta ~ U[0.5, 2],
    cube centroids of side N^(1/3) (mean spacing 1), jitter 0.3.  System i
    draws from SeedSequence(seed).spawn(S)[i]."""
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(S)):
        rng = np.random.default_rng(ss)
        N = int(rng.integers(n_lo, n_hi + 1))
        P = int(rng.choice([16, 32, 64]))
        beta = float(rng.uniform(0.5, 2.0))
        side = N ** (1.0 / 3.0)
        c = rng.uniform(0.0, side, size=(N, 3))
        R = c[:, None, :] + rng.normal(0.0, 0.3, size=(N, P, 3))
        out.append(System(R, beta=beta, name="batch[%d] N%d P%d" % (i, N, P)))
    return out


def config_large(seed=5) -> System:
    """N=4096, P=64, beta=1, periodic cube of side 16 (minimum image),
    uniform centroids, bead jitter 0.25."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 16.0, size=(4096, 3))
    R = c[:, None, :] + rng.normal(0.0, 0.25, size=(4096, 64, 3))
    return System(R, beta=1.0, box=16.0, name="large N4096 P64 periodic L16")


def initial_velocities(N: int, P: int, beta: float, m: float, seed):
    """Maxwell-Boltzmann draw N(0, 1/(m beta)) per bead and component, (N, P, 3)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, math.sqrt(1.0 / (m * beta)), size=(N, P, 3))
