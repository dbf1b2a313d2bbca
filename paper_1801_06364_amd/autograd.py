"""torch.autograd binding of the checkpointed discrete adjoint.

``RteSolve.apply(mu_a, mu_s, problem)`` returns the detector readings
``[steps][n_det]`` of a forward solve on the GPU (through the C-ABI); its
backward returns dJ/dmu_a and dJ/dmu_s from ``rte_adjoint`` (exact reverse
mode of the discrete RK4 scheme, stage states recomputed from sqrt(T)
checkpoints). ``problem`` is a dict with the fixed inputs: n, N, dx, c, dt,
g, psi0, q, W, mu0, mu1, precision, det_index, steps, and optionally every
(checkpoint interval) and stream.
"""
from __future__ import annotations

import numpy as np
import torch

from .rte import Solver


class RteSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu_a: torch.Tensor, mu_s: torch.Tensor, problem: dict):
        p = dict(problem)
        steps = int(p.pop("steps"))
        every = int(p.pop("every", 0))
        solver = Solver(mu_a=mu_a.detach().cpu().double().numpy(),
                        mu_s=mu_s.detach().cpu().double().numpy(), record_steps=steps, **p)
        solver.forward_checkpointed(steps, every)
        readings = torch.from_numpy(solver.readings().copy())
        ctx.solver = solver
        ctx.devtype = (mu_a.device, mu_a.dtype)
        return readings.to(device=mu_a.device, dtype=mu_a.dtype)

    @staticmethod
    def backward(ctx, grad_readings: torch.Tensor):
        solver = ctx.solver
        ga, gs = solver.adjoint(grad_readings.detach().cpu().double().numpy())
        solver.close()
        ctx.solver = None
        dev, dt = ctx.devtype
        return (torch.from_numpy(ga).to(device=dev, dtype=dt),
                torch.from_numpy(gs).to(device=dev, dtype=dt), None)


def rte_solve(mu_a: torch.Tensor, mu_s: torch.Tensor, problem: dict) -> torch.Tensor:
    """Detector readings as a differentiable function of mu_a and mu_s."""
    return RteSolve.apply(mu_a, mu_s, problem)
