"""Driver loop of the hot path: neighbour build -> NEP forces -> integrator.

One stream, no per-step host synchronisation: the sticky device flags of
the neighbour lists and of the force workspace are polled every
`check_every` steps.  The step is the paper's workflow (Sec. II.A): thermostat,
half kick, free ring-polymer step, forces, half kick, thermostat; the two
integrator halves around consecutive force evaluations run as one fused
launch.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import inputs as I
from . import lib


def default_capacity(rc: float, density: float, n_species: int, slack: float = 1.6) -> int:
    """First guess of a candidate row length from the mean density (refitted after one build)."""
    n = density * 4.0 / 3.0 * math.pi * rc ** 3
    return int(math.ceil(n * slack)) + 8


class NepPimd:
    """NEP forces for P beads of one periodic system plus the ring-polymer integrator."""

    def __init__(self, model_path: str, system: I.System, *, dt: float, T: float, tau: float = 100.0,
                 mode: str = "trpmd", seed: int = 0, caps: Optional[tuple] = None, check_every: int = 50,
                 want_atom: bool = False, skin: float = 0.5):
        import torch
        self.torch = torch
        dev = torch.device("cuda")
        self.model = lib.Model(model_path)
        self.P, self.N = system.P, system.N
        self.box = np.asarray(system.box, np.float64)
        self.pos = torch.tensor(system.pos, dtype=torch.float64, device=dev)
        self.vel = torch.tensor(system.vel, dtype=torch.float64, device=dev)
        self.types = torch.tensor(system.types, dtype=torch.int32, device=dev)
        self.mass = torch.tensor(system.masses, dtype=torch.float64, device=dev)
        self.F = torch.zeros((self.P, self.N, 3), dtype=torch.float32, device=dev)
        self.E = torch.zeros(self.P, dtype=torch.float64, device=dev)
        self.W = torch.zeros((self.P, 9), dtype=torch.float64, device=dev)
        self.E_atom = torch.zeros((self.P, self.N), dtype=torch.float32, device=dev) if want_atom else None
        self.W_atom = torch.zeros((self.P, self.N, 9), dtype=torch.float32, device=dev) if want_atom else None
        dens = self.N / float(np.prod(self.box))
        S = self.model.n_species
        rcR, rcA = self.model.rc_radial, self.model.rc_angular
        self.caps = tuple(caps) if caps else (default_capacity(rcR + 0.5, dens, S), default_capacity(rcR, dens, S),
                                              default_capacity(rcA, dens, S))
        self.nl = None
        self.skin = skin
        self.ws = lib.Workspace(self.model, self.P, self.N)
        self.pimd = lib.Pimd(self.P, self.N, self.mass, dt, T, tau, mode, seed)
        self.check_every = check_every
        self.step_no = 0
        self.started = False
        self.graph = None
        self.step_dev = None
        self._fit_capacity()

    # ------------------------------------------------------------------
    def _fit_capacity(self):
        """Size the candidate rows to the starting configuration (slack for the run)."""
        self.nl = lib.fitted_neighbor_list(self.model, self.pos, self.box, self.types, *self.caps, skin=self.skin)
        self.caps = self.nl.caps

    def forces(self):
        """Neighbour lists + NEP energy, forces and virial at the current positions."""
        self.nl.build(self.pos, self.box, self.types)
        self.ws.compute(self.nl, self.pos, self.box, self.types, self.E, self.F, self.W, self.E_atom, self.W_atom)

    def check(self):
        """Poll the sticky flags (synchronises); raise on overflow or non-finite values."""
        st = self.nl.status(clear=True)
        flags, mr, ma = st["flags"], st["max_radial"], st["max_angular"]
        if flags & lib.FLAG_NEIGHBOR_OVERFLOW:
            raise lib.NepError(5, f"list overflow: need {st['max_candidates']}/{mr}/{ma}, capacities {self.caps}")
        wf = self.ws.poll(clear=True)
        if (flags | wf) & lib.FLAG_NONFINITE:
            raise lib.NepError(6, "non-finite force or position")
        if (flags | wf) & lib.FLAG_BAD_TYPE:
            raise lib.NepError(1, "species index outside the model's range")
        return mr, ma

    def start(self):
        self.forces()
        self.pimd.step(self.pos, self.vel, self.F, self.step_no, lib.PRE)
        self.started = True

    def step(self):
        """One full step: forces at the advanced positions, then POST(n) + PRE(n+1)."""
        if self.graph is not None:
            self.graph.replay()
        else:
            if not self.started:
                self.start()
            self.forces()
            self.pimd.step(self.pos, self.vel, self.F, self.step_no, lib.FUSED)
        self.step_no += 1
        if self.check_every and self.step_no % self.check_every == 0:
            self.check()

    def run(self, n: int):
        for _ in range(n):
            self.step()

    def capture(self):
        """Capture one full step (lists, forces, fused integrator stage) as a HIP graph.

        The step number then lives in a device counter advanced by the graph
        itself, so every replay draws fresh noise.  The box and the species
        must stay fixed while the graph is in use; `release()` returns to
        eager launches."""
        t = self.torch
        if not self.started:
            self.start()
        # one eager step first so that every lazy allocation has happened
        self.step()
        self.step_dev = t.tensor([self.step_no], dtype=t.int64, device=self.pos.device)
        t.cuda.synchronize()
        g = t.cuda.CUDAGraph()
        with t.cuda.graph(g):
            self.nl.build(self.pos, self.box, self.types)
            self.ws.compute(self.nl, self.pos, self.box, self.types, self.E, self.F, self.W, self.E_atom, self.W_atom)
            self.pimd.step_dev(self.pos, self.vel, self.F, self.step_dev, lib.FUSED)
        t.cuda.synchronize()
        # capture does not execute: the counter and the state are unchanged
        self.graph = g

    def release(self):
        self.graph = None

    def finish(self):
        """Close the current step (forces + POST), leaving synchronised q and v."""
        self.graph = None
        if not self.started:
            self.start()
        self.forces()
        self.pimd.step(self.pos, self.vel, self.F, self.step_no, lib.POST)
        self.started = False
        self.step_no += 1
