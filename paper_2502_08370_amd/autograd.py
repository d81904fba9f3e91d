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
        u64 = u0.detach().to(device=problem.device, dtype=torch.float64).reshape(-1).contiguous()
        th64 = theta.detach().to(device=problem.device, dtype=torch.float64).reshape(-1).contiguous()
        problem.set_coefficients(0, th64)
        U = problem.new_states()
        problem.sequential_fine(u64, U)
        ctx.problem = problem
        ctx.u_meta = (u0.shape, u0.dtype, u0.device)
        ctx.th_meta = (theta.shape, theta.dtype, theta.device)
        ctx.save_for_backward(u64, th64)
        npts = ins["nx"] * ins["ny"]
        return U[-npts:].view(shape).clone()

    @staticmethod
    def backward(ctx, gT):
        u64, th64 = ctx.saved_tensors
        problem = ctx.problem
        problem.set_coefficients(0, th64)
        g0 = torch.empty_like(u64)
        gth = torch.empty_like(th64)
        lam = gT.detach().to(device=problem.device, dtype=torch.float64).reshape(-1).contiguous()
        problem.adjoint(u64, lam, g0, gth)
        (us, ud, udev), (ts, td, tdev) = ctx.u_meta, ctx.th_meta
        return g0.view(us).to(device=udev, dtype=ud), gth.view(ts).to(device=tdev, dtype=td), None


def fine_map(u0, theta, problem):
    return FineMap.apply(u0, theta, problem)
