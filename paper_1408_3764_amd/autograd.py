"""Differentiable total energy: torch.autograd.Function over the library's
total-energy and gradient kernels.

U(positions, eps, sigma) = U_pair + U_tail of one box (Eq. 1 truncated at rc,
plus the tail correction).  Forward uploads the positions and the force field
into the box and runs gcmc_total_energy; backward runs gcmc_backward, which
returns dU/dr_i (forces are its negative, e.g. for force-biased proposals) and
dU/d eps_ab, dU/d sigma_ab (for force-field fitting), the cutoff held fixed.
The gradient with respect to the symmetric tables splits an unordered species
pair a != b half into [a][b] and half into [b][a].
"""
from __future__ import annotations

import torch

from .box import Box


class LJEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos: torch.Tensor, eps: torch.Tensor, sigma: torch.Tensor, box: Box):
        if pos.dtype != torch.float64 or not pos.is_cuda:
            raise TypeError("positions must be a float64 device tensor")
        box.set_params(eps.detach().cpu().numpy(), sigma.detach().cpu().numpy())
        box.set_positions_device(pos.detach())
        U = box.total_energy_device()
        ctx.box = box
        ctx.n = pos.shape[0]
        ctx.version = box.version
        ctx.save_for_backward(pos.detach(), eps.detach(), sigma.detach())
        return U[0] + U[1]

    @staticmethod
    def backward(ctx, gU):
        box = ctx.box
        if box.version != ctx.version:
            # the box was changed after this forward (another forward, new parameters, moves):
            # the gradient is taken at the saved inputs, put back into the box
            pos, eps, sigma = ctx.saved_tensors
            box.set_params(eps.cpu().numpy(), sigma.cpu().numpy())
            box.set_positions_device(pos)
        g, de, ds = box.backward_device(ctx.n)
        return gU * g, gU * de, gU * ds, None


def lj_energy(pos: torch.Tensor, eps: torch.Tensor, sigma: torch.Tensor, box: Box) -> torch.Tensor:
    """Total energy of `box` at `pos` with pair tables eps, sigma (differentiable in all three)."""
    return LJEnergy.apply(pos, eps, sigma, box)
