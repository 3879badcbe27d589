"""torch.autograd wrapper of the FDTD objective (arXiv 2412.12360, section 2.2).

forward: write eps_r of the design box into the solver's material, run the
full forward solve with the interface record, return J.  backward: the
time-reversed adjoint pass of libfdtd returns dJ/deps_r over the design box.
The map from design parameters to eps_r (for example eps_r = 2.25 + 10 rho)
stays in plain torch, so autograd supplies its derivative.
"""
from __future__ import annotations

import torch


class FdtdObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_design: torch.Tensor, solver) -> torch.Tensor:
        pr = solver.prob
        if tuple(eps_design.shape) != pr.design_shape():
            raise ValueError(f"eps_design shape {tuple(eps_design.shape)} != design box {pr.design_shape()}")
        inv = solver.inv_eps.clone()
        inv[pr.design_slices()] = 1.0 / eps_design.detach().to(torch.float32)
        solver.reset()
        solver.set_inv_eps(inv)
        _, J = solver.forward()
        ctx.solver = solver
        return J.clone().reshape(())

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        g, _ = ctx.solver.grad()
        return gJ * g, None


def objective(eps_design: torch.Tensor, solver) -> torch.Tensor:
    """J(eps_design) with dJ/deps from the time-reversal adjoint."""
    return FdtdObjective.apply(eps_design, solver)
