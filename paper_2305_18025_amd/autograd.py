"""V^[1,N] as a differentiable PyTorch function.

forward  : interior springs + forward recursion (pimdb_exchange_energy_save),
           keeping the forward potentials and forward-weighted endpoint
           displacements in a per-call state buffer;
backward : the adjoint kernel (pimdb_exchange_adjoint) -- the paper's force
           evaluation: backward recursion, connection probabilities and the
           exterior/interior bead forces, scaled by the incoming gradient.
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from .core import BosonicExchange


class _ExchangePotential(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos: torch.Tensor, engine: BosonicExchange):
        energy = torch.empty(engine.S, dtype=torch.float64, device=engine.device)
        state = torch.empty(engine.state_bytes(), dtype=torch.uint8, device=engine.device)
        engine.energy_save(pos, state, energy)
        ctx.save_for_backward(pos)
        ctx.state = state
        ctx.engine = engine
        return energy

    @staticmethod
    @once_differentiable
    def backward(ctx, grad_energy: torch.Tensor):
        (pos,) = ctx.saved_tensors
        engine = ctx.engine
        grad = engine.empty()
        engine.adjoint(pos, ctx.state, grad_energy.contiguous().to(torch.float64), grad)
        return grad, None


def exchange_potential(pos: torch.Tensor, engine: BosonicExchange) -> torch.Tensor:
    """Energies V^[1,N] (one per system) of packed positions, differentiable
    with respect to ``pos``."""
    return _ExchangePotential.apply(pos, engine)
