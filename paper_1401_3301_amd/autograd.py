"""torch.autograd wrapper around the assembly and its adjoint.

``BilinearAssembly.apply(q, w, a, b, plan)`` returns the scalar
J = a^T (S(q) + M_w(q)) b, where S is the P1 stiffness matrix and M_w the
weighted mass matrix of the mesh behind ``plan`` (Sections 4.1-4.2 of the
paper).  Its backward calls the hand-written adjoint kernel
(``fem_assemble_backward``) for dJ/dq and dJ/dw, the shape derivative through
the element Jacobians; a and b are treated as constants (no gradient).
"""
from __future__ import annotations

import torch

from . import femasm


class BilinearAssembly(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, w, a, b, plan):
        if not isinstance(plan, femasm.Plan):
            raise TypeError("plan must be a femasm.Plan")
        q = q.detach().contiguous()
        w = w.detach().contiguous()
        a = a.detach().contiguous()
        b = b.detach().contiguous()
        vs = plan.numeric("STIFF", q)
        vm = plan.numeric("MASS_W", q, w)
        js = plan.bilinear("STIFF", vs, a, b)
        jm = plan.bilinear("MASS_W", vm, a, b)
        ctx.plan = plan
        ctx.save_for_backward(q, w, a, b)
        return (js + jm).reshape(())

    @staticmethod
    def backward(ctx, gJ):
        q, w, a, b = ctx.saved_tensors
        need_q, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gw, gq = ctx.plan.backward(q, w, a, b, want_w=need_w, want_q=need_q)
        gq = gq * gJ if gq is not None else None
        gw = gw * gJ if gw is not None else None
        return gq, gw, None, None, None


def bilinear_energy(q, w, a, b, plan):
    """J = a^T (S(q) + M_w(q)) b, differentiable in q and w."""
    return BilinearAssembly.apply(q, w, a, b, plan)
