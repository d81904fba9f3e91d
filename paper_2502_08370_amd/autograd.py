"""torch.autograd front end of the adjoint (pr_adjoint).

FineMap.apply(u0, theta, problem) returns u(T) = (F^s)^N u0, the fine map of
section 3 (parareal's fixed point), for a single-instance 2D dimensional-
splitting handle created with a nodal log coefficient (theta). The forward
sets the coefficient (refactorising every line system) and runs the
sequential fine solve on the GPU; backward calls pr_adjoint with lambda_T =
the incoming gradient and returns dL/du0 and dL/dtheta.
"""
from __future__ import annotations

import torch

from . import Problem

__all__ = ["FineMap", "fine_map"]


class FineMap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, theta, problem: Problem):
        ins = problem.instances[0]
        shape = (ins["ny"], ins["nx"])
        problem.set_coefficients(0, theta)
        U = problem.new_states()
        problem.sequential_fine(u0.reshape(-1).contiguous(), U)
        ctx.problem = problem
        ctx.save_for_backward(u0, theta)
        npts = ins["nx"] * ins["ny"]
        return U[-npts:].view(shape).clone()

    @staticmethod
    def backward(ctx, gT):
        u0, theta = ctx.saved_tensors
        problem = ctx.problem
        problem.set_coefficients(0, theta)
        g0 = torch.empty_like(u0, dtype=torch.float64).reshape(-1)
        gth = torch.empty_like(theta, dtype=torch.float64).reshape(-1)
        problem.adjoint(u0.reshape(-1).contiguous(), gT.reshape(-1).contiguous().double(), g0, gth)
        return g0.view(u0.shape), gth.view(theta.shape), None


def fine_map(u0, theta, problem):
    return FineMap.apply(u0, theta, problem)
