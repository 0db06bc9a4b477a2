"""PyTorch autograd wrapper: E = REANN(pos) with forces from the library's hand-written
adjoint kernels (the chain rule of Sec. 2.2, Eqs. (3)-(5)), not from torch autograd.

PyTorch supplies only device memory and the stream; both passes run in the library.
"""
from __future__ import annotations

import torch

from ._binding import Plan, ReannError

REANN_E_STATE = -7


class _REANNEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos: torch.Tensor, plan: Plan):
        pos = pos.detach().contiguous()
        energy = torch.empty((), dtype=torch.float64, device=pos.device)
        plan.forward(pos, energy)
        ctx.plan = plan
        # the plan keeps the state of its latest forward only; the backward checks that no
        # other forward has run on it since this one
        ctx.generation = plan.generation()
        ctx.n = pos.shape[0]
        ctx.device = pos.device
        return energy

    @staticmethod
    def backward(ctx, grad_energy: torch.Tensor):
        if ctx.plan.generation() != ctx.generation:
            raise ReannError(REANN_E_STATE, "backward of a REANN energy whose plan has run another forward since: "
                                            "the plan holds only its latest forward's state (use one plan per "
                                            "energy that is kept for a backward)")
        g = grad_energy.detach().to(torch.float64).contiguous().reshape(())
        forces = torch.empty((ctx.n, 3), dtype=torch.float64, device=ctx.device)
        ctx.plan.backward(forces, grad_energy=g)
        return -forces, None


def reann_energy(pos: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Total energy (eV, float64 scalar tensor) of the plan's system at ``pos``; its
    gradient w.r.t. ``pos`` is -F.  A backward must follow the plan's latest forward: a
    backward after another forward on the same plan raises ReannError (REANN_E_STATE)."""
    return _REANNEnergy.apply(pos, plan)
