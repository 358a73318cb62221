"""NEP energy as a differentiable torch function of the bead positions.

The forward pass is `neighbor_build` + `nep_compute` on the current stream;
the backward pass needs no further kernel, because `nep_compute` already is
the adjoint of the energy: it returns F = -dE/dpos for every bead (Sec. II.A,
forces from the site energies of Sec. II.C).  For an upstream gradient gE of
the per-bead energies the position gradient is therefore -gE[b] * F[b].
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import lib


class NepCalculator:
    """Model, neighbour lists and workspace for P beads of one periodic system."""

    def __init__(self, model_path: str, P: int, N: int, box, types, *, pos_hint=None, skin: float = 0.0):
        import torch
        self.torch = torch
        self.model = lib.Model(model_path)
        self.P, self.N = int(P), int(N)
        self.box = np.asarray(box, np.float64)
        self.types = torch.as_tensor(np.asarray(types), dtype=torch.int32, device="cuda").contiguous()
        self.ws = lib.Workspace(self.model, self.P, self.N)
        self.skin = skin
        self.nl: Optional[lib.NeighborList] = None
        if pos_hint is not None:
            self._fit(self._pos(pos_hint))

    def _pos(self, pos):
        t = self.torch
        p = pos.detach()
        if p.dtype != t.float64 or not p.is_cuda or not p.is_contiguous():
            p = p.to(device="cuda", dtype=t.float64).contiguous()
        if tuple(p.shape) != (self.P, self.N, 3):
            raise ValueError(f"positions must have shape {(self.P, self.N, 3)}, got {tuple(p.shape)}")
        return p

    def _fit(self, p):
        dens = self.N / float(np.prod(self.box))
        rc = self.model.rc_radial
        n = dens * 4.0 / 3.0 * np.pi
        caps = (int(n * (rc + 0.5 + self.skin) ** 3 * 1.6) + 8,
                int(n * (self.model.rc_angular + 0.5 + self.skin) ** 3 * 1.6) + 8)
        self.nl = lib.fitted_neighbor_list(self.model, p, self.box, self.types, *caps, skin=self.skin)

    def evaluate(self, pos, want_virial: bool = False):
        """E [P] float64, F [P,N,3] float32 (and W [P,9] float64) at pos; raises on device flags."""
        t = self.torch
        p = self._pos(pos)
        if self.nl is None:
            self._fit(p)
        E = t.empty(self.P, dtype=t.float64, device="cuda")
        F = t.empty((self.P, self.N, 3), dtype=t.float32, device="cuda")
        W = t.empty((self.P, 9), dtype=t.float64, device="cuda")
        self.nl.build(p, self.box, self.types)
        self.ws.compute(self.nl, p, self.box, self.types, E, F, W)
        st = self.nl.status(clear=True)
        if st["flags"] & lib.FLAG_NEIGHBOR_OVERFLOW:
            self._fit(p)   # lists grew: refit and evaluate again
            return self.evaluate(pos, want_virial)
        if st["flags"] or self.ws.poll(clear=True):
            raise lib.NepError(6, f"device flags {st['flags']:#x} raised during the NEP evaluation")
        return (E, F, W) if want_virial else (E, F)


class NepEnergy:
    """torch.autograd.Function: E[P] = NEP(pos[P,N,3]); backward uses the hand-written adjoint."""

    _fn = None

    @classmethod
    def apply(cls, pos, calc: NepCalculator):
        if cls._fn is None:
            cls._fn = _make_function()
        return cls._fn.apply(pos, calc)


def _make_function():
    import torch

    class _NepEnergyFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, pos, calc):
            E, F = calc.evaluate(pos)
            ctx.save_for_backward(F)
            ctx.in_dtype = pos.dtype
            return E.to(pos.dtype) if pos.dtype != torch.float64 else E

        @staticmethod
        def backward(ctx, gE):
            (F,) = ctx.saved_tensors
            g = -(F.to(torch.float64) * gE.to(torch.float64)[:, None, None])
            return g.to(ctx.in_dtype), None

    return _NepEnergyFn


def nep_energy(pos, calc: NepCalculator):
    """Differentiable per-bead NEP energies of pos [P,N,3]."""
    return NepEnergy.apply(pos, calc)
