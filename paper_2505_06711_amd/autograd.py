"""PyTorch autograd wrapper: E = REANN(pos) with forces from the library's hand-written
adjoint kernels (the chain rule of Sec. 2.2, Eqs. (3)-(5)), not from torch autograd.

PyTorch supplies only device memory and the stream; both passes run in the library.
"""
from __future__ import annotations

import torch

from ._binding import Plan


class _REANNEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos: torch.Tensor, plan: Plan):
        pos = pos.detach().contiguous()
        energy = torch.empty((), dtype=torch.float64, device=pos.device)
        plan.forward(pos, energy)
        ctx.plan = plan
        ctx.n = pos.shape[0]
        ctx.device = pos.device
        return energy

    @staticmethod
    def backward(ctx, grad_energy: torch.Tensor):
        g = grad_energy.detach().to(torch.float64).contiguous().reshape(())
        forces = torch.empty((ctx.n, 3), dtype=torch.float64, device=ctx.device)
        ctx.plan.backward(forces, grad_energy=g)
        return -forces, None


def reann_energy(pos: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Total energy (eV, float64 scalar tensor) of the plan's system at ``pos``; its
    gradient w.r.t. ``pos`` is -F.  One backward per forward."""
    return _REANNEnergy.apply(pos, plan)
