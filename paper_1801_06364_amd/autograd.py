"""torch.autograd binding of the checkpointed discrete adjoint.

``rte_solve(mu_a, mu_s, problem)`` returns the detector readings
``[steps][n_det]`` of a forward solve on the GPU (through the C-ABI); its
backward returns dJ/dmu_a and dJ/dmu_s from the exact reverse mode of the
discrete RK4 scheme (stage states recomputed from sqrt(T) checkpoints).
``problem`` is an :class:`RteProblem`, or a dict with the fixed inputs (n, N,
dx, c, dt, g, psi0, q, W, mu0, mu1, precision, det_index, steps, and
optionally every and stream), turned into one on first use and kept in the
dict.

Everything stays on the device: the problem holds one solver handle (created
once) and the initial state as a CUDA tensor; every forward call loads the
CUDA maps mu_a, mu_s into the handle (loss maps rebuilt on the device),
resets the state, runs the checkpointed forward solve and copies the
readings device to device; the backward passes the CUDA adjoint sources and
receives CUDA gradients.
"""
from __future__ import annotations

import numpy as np
import torch

from .rte import Solver


class RteProblem:
    """The fixed part of a differentiable solve: one device-resident solver
    (maps replaced per call) and its initial state on the device."""

    def __init__(self, n, N, dx, c, dt, g, psi0=None, q=None, W=0, mu0=0.01, mu1=1.0,
                 precision="f32", det_index=None, steps=1, every=0, stream=None, device="cuda"):
        self.n, self.N, self.steps, self.every = int(n), int(N), int(steps), int(every)
        zeros = np.zeros((n, n, n))
        # created once with placeholder maps; each solve loads its own
        self.solver = Solver(n, N, dx, c, dt, zeros, zeros, g, psi0=psi0, q=q, W=W, mu0=mu0, mu1=mu1,
                             precision=precision, det_index=det_index, record_steps=self.steps,
                             stream=stream, device=device)
        m = 0 if psi0 is None else np.asarray(psi0).size // n ** 3
        self.psi0 = (torch.from_numpy(np.ascontiguousarray(psi0, np.float64).reshape(-1)).to(device)
                     if m else torch.zeros(0, dtype=torch.float64, device=device))

    def forward(self, mu_a: torch.Tensor, mu_s: torch.Tensor) -> torch.Tensor:
        s = self.solver
        s.set_medium_device(mu_a.detach().to(torch.float64).contiguous().view(-1),
                            mu_s.detach().to(torch.float64).contiguous().view(-1))
        s.set_state_device(self.psi0)
        s.forward_checkpointed(self.steps, self.every)
        return s.readings_device().clone()

    def backward(self, grad_readings: torch.Tensor):
        return self.solver.adjoint_device(grad_readings.detach())

    def close(self):
        self.solver.close()


def _problem_of(problem) -> RteProblem:
    if isinstance(problem, RteProblem):
        return problem
    p = problem.get("_rte_problem")
    if p is None:
        args = {k: v for k, v in problem.items() if not k.startswith("_")}
        p = problem["_rte_problem"] = RteProblem(**args)
    return p


class RteSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu_a: torch.Tensor, mu_s: torch.Tensor, problem):
        p = _problem_of(problem)
        ctx.problem = p
        ctx.devtype = (mu_a.device, mu_a.dtype)
        r = p.forward(mu_a, mu_s)
        return r.to(device=mu_a.device, dtype=mu_a.dtype)

    @staticmethod
    def backward(ctx, grad_readings: torch.Tensor):
        ga, gs = ctx.problem.backward(grad_readings)
        ctx.problem = None
        dev, dt = ctx.devtype
        return ga.to(device=dev, dtype=dt), gs.to(device=dev, dtype=dt), None


def rte_solve(mu_a: torch.Tensor, mu_s: torch.Tensor, problem) -> torch.Tensor:
    """Detector readings as a differentiable function of mu_a and mu_s."""
    return RteSolve.apply(mu_a, mu_s, problem)
