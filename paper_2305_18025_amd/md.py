"""Velocity-Verlet molecular dynamics with the bosonic exchange forces,
optionally captured in a HIP graph (torch.cuda.CUDAGraph).

One step (pimdb_md_step): v += dt/(2m) F;  x += dt v;  F <- exchange forces
(+ trap);  v += dt/(2m) F.  Each bead moves with the particle mass m.
"""
from __future__ import annotations

import torch

from .core import BosonicExchange


class VelocityVerlet:
    def __init__(self, engine: BosonicExchange, pos: torch.Tensor, vel: torch.Tensor, dt: float):
        self.engine = engine
        self.pos = pos
        self.vel = vel
        self.dt = float(dt)
        self.forces = engine.empty()
        self.energy = torch.empty(engine.S, dtype=torch.float64, device=engine.device)
        engine.forces(self.pos, out=self.forces, energy=self.energy)
        self.graph = None
        self.graph_steps = 0

    def step(self, n: int = 1):
        for _ in range(n):
            self.engine.md_step(self.pos, self.vel, self.forces, self.energy, self.dt)

    def capture(self, steps_per_replay: int = 1):
        """Record `steps_per_replay` steps into one graph (no allocation,
        host synchronisation or host reads happen inside)."""
        side = torch.cuda.Stream(device=self.engine.device)
        side.wait_stream(torch.cuda.current_stream(self.engine.device))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                for _ in range(steps_per_replay):
                    self.engine.md_step(self.pos, self.vel, self.forces, self.energy, self.dt)
        torch.cuda.current_stream(self.engine.device).wait_stream(side)
        self.graph = g
        self.graph_steps = steps_per_replay
        return g

    def replay(self, n: int = 1):
        for _ in range(n):
            self.graph.replay()

    def kinetic(self) -> torch.Tensor:
        """Kinetic energy per system, sum 1/2 m v^2 over beads (torch reduction)."""
        out = []
        for s in range(self.engine.S):
            v = self.engine.view(self.vel, s)
            out.append(0.5 * self.engine.m[s] * (v * v).sum())
        return torch.stack(out)
