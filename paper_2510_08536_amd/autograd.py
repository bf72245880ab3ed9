"""Adjoint of the repartitioned solve as a torch.autograd.Function.

forward:  update the plan with the slot values, solve A x = b (FP64 PCG or
          mixed refinement), keep x (not the Krylov history).
backward: lambda = A^-T dL/dx by one more solve (opts.transpose = 1: with CG,
          A is symmetric and this is the same system; with BiCGStab the
          library gathers A^T's values on the same pattern), dL/db = lambda,
          and the slot gradient
          dL/dv_k = -lambda[row(k)] x[col(k)] from rp_value_grad, returned in
          receive-buffer order.  The caller's own assembly (face coefficient ->
          slot values) chains these to its parameters through torch.
"""
from __future__ import annotations

import torch

from .rp import Plan, default_opts, rp_solve_opts


class RepartSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, slot_values: torch.Tensor, b: torch.Tensor, plan: Plan, opts=None):
        slot_values = slot_values.contiguous()
        o = opts if opts is not None else default_opts()
        o = rp_solve_opts.from_buffer_copy(o)     # the caller's options stay untouched
        o.transpose = 0
        plan.update_slots(slot_values)
        x, info = plan.solve(b.contiguous(), opts=o)
        ctx.plan = plan
        ctx.version = plan.version
        ctx.opts = o
        ctx.info = info
        ctx.save_for_backward(slot_values, x)
        return x

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        slot_values, x = ctx.saved_tensors
        plan = ctx.plan
        if plan.version != ctx.version:
            # the plan was refreshed with other values since the forward pass
            plan.update_slots(slot_values)
        o = rp_solve_opts.from_buffer_copy(ctx.opts)
        o.x0_zero = 1
        o.transpose = 1
        lam, _ = plan.solve(gx.contiguous(), opts=o)
        g_slots = plan.value_grad(lam, x) if ctx.needs_input_grad[0] else None
        g_b = lam if ctx.needs_input_grad[1] else None
        return g_slots, g_b, None, None


def repart_solve(slot_values, b, plan: Plan, opts=None):
    return RepartSolve.apply(slot_values, b, plan, opts)
