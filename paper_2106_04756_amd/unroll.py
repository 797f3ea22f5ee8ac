"""Differentiable unrolled PDHG: torch.autograd.Function over pdlp_unroll_forward/backward.

    x_T, y_T = unrolled_pdhg(solver, c, q, steps=500, segment=50)
    loss = ((x_T - x_tgt) ** 2).sum(); loss.backward()      # fills c.grad, q.grad

The forward and the adjoint both run in libpdlp_hip.so: T fixed steps of Eq. (3) on the
solver's preconditioned LP (eta, omega, D1, D2 frozen, no restarts or rejections), then the
hand-written reverse pass (transposed products times the projection masks).  This module only
allocates the output tensors and passes pointers.
"""
from __future__ import annotations

import torch

from .pdlp import Solver


class UnrolledPDHG(torch.autograd.Function):
    """(c, q) -> (x_T, y_T) of the solver's LP with objective c and right-hand side q."""

    @staticmethod
    def forward(ctx, c, q, solver: Solver, steps: int, segment: int, eta: float, omega: float):
        c = c.detach().to(torch.float64).contiguous()
        q = q.detach().to(torch.float64).contiguous()
        x = torch.empty(solver.n, dtype=torch.float64, device=c.device)
        y = torch.empty(solver.m, dtype=torch.float64, device=c.device)
        solver.unroll_forward(c, q, steps, segment, eta, omega, x, y)
        info = solver.unroll_info()
        ctx.solver = solver
        ctx.args = (steps, segment, info["eta"], info["omega"])
        ctx.tape = solver.unroll_id
        ctx.save_for_backward(c, q)
        return x, y

    @staticmethod
    def backward(ctx, gx, gy):
        solver = ctx.solver
        c, q = ctx.saved_tensors
        if solver.unroll_id != ctx.tape:
            # another forward ran on this solver since: replay this one (deterministic kernels
            # give the same trajectory and masks)
            steps, segment, eta, omega = ctx.args
            solver.unroll_forward(c, q, steps, segment, eta, omega, None, None)
        gc = torch.empty_like(c)
        gq = torch.empty_like(q)
        gx = None if gx is None else gx.to(torch.float64).contiguous()
        gy = None if gy is None else gy.to(torch.float64).contiguous()
        solver.unroll_backward(gx, gy, gc, gq)
        ctx.tape = solver.unroll_id
        return gc, gq, None, None, None, None, None


def unrolled_pdhg(solver: Solver, c, q, steps: int = 500, segment: int = 50, eta: float = 0.0,
                  omega: float = 0.0):
    """x_T, y_T after `steps` PDHG steps (user units); differentiable in c and q.
    eta <= 0: 0.9 / ||K~||_2; omega <= 0: the LP's initial primal weight."""
    return UnrolledPDHG.apply(c, q, solver, steps, segment, eta, omega)
