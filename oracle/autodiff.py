"""Forward recurrence in torch CPU float64, differentiated by autograd
(TEST INFRASTRUCTURE).

V^[1,N] is computed from the recurrence over cycle lengths (Background,
recurrence for V^[1,N], with V^[1,0] = 0) using log-sum-exp.  The cycle
energies use the closed form obtained by unrolling the paper's incremental
recurrence (Theory, "Reducing the potential"): the interior energies of
particles u..v, the links from the last bead of l to the first bead of l+1
for l = u..v-1, and the closing spring from the last bead of v to the first
bead of u.  The forces are -dV/dR from autograd; they do not use the
connection probabilities at all, so they check the probabilistic force
expressions independently.
"""
from __future__ import annotations

import numpy as np
import torch


def _mi(d, L):
    if L > 0:
        return d - L * torch.round(d / L)  # half to even, zero gradient
    return d


def potential(Rt, beta, m, omegaP, L=0.0):
    """V^[1,N] as a differentiable torch scalar; Rt is (N, P, 3) float64."""
    N, P, _ = Rt.shape
    k = 0.5 * m * omegaP ** 2
    dint = _mi(Rt[:, 1:, :] - Rt[:, :-1, :], L)
    eint = k * (dint * dint).sum(dim=(1, 2))  # (N,)
    zero = torch.zeros(1, dtype=Rt.dtype)
    ci = torch.cat([zero, torch.cumsum(eint, 0)])  # ci[v] = sum_{l<=v} E_int
    if N > 1:
        dl = _mi(Rt[:-1, -1, :] - Rt[1:, 0, :], L)
        link = k * (dl * dl).sum(dim=1)  # link[l-1] = spring l -> l+1
        cl = torch.cat([zero, torch.cumsum(link, 0)])  # cl[v] = sum_{l<=v} link
    else:
        cl = zero
    dc = _mi(Rt[:, -1, None, :] - Rt[None, :, 0, :], L)  # [v-1, u-1]
    s = k * (dc * dc).sum(dim=2)
    vf = [torch.zeros((), dtype=Rt.dtype)]
    for v in range(1, N + 1):
        u = torch.arange(1, v + 1)
        e_uv = (ci[v] - ci[u - 1]) + (cl[v - 1] - cl[u - 1]) + s[v - 1, u - 1]
        prev = torch.stack(vf)  # V^[1, u-1] for u = 1..v
        x = -beta * (prev + e_uv)
        vf.append(-(torch.logsumexp(x, 0) - np.log(v)) / beta)
    return vf[-1]


def exchange(R, beta, m, omegaP, L=0.0):
    """Returns (V, F) with F = -dV/dR in the (N, P, 3) layout."""
    Rt = torch.tensor(np.asarray(R, dtype=np.float64), requires_grad=True)
    V = potential(Rt, beta, m, omegaP, L)
    (g,) = torch.autograd.grad(V, Rt)
    return float(V.detach()), (-g).numpy()
