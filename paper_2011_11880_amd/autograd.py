"""Differentiable residual: F(x; p) as a torch.autograd.Function whose
backward is libpf's adjoint kernel (pf_vjp).

    F = PFResidual.apply(x, params, plan)

``params`` is the device vector [r(B), x(B), b(B), tap(B), shift_deg(B),
load_p(N_L), load_q(N_L)] (api.params_vector builds it).  The forward loads it into the
plan (pf_set_params, a device kernel) and evaluates the residual; backward
returns (J^T w, (dF/dp)^T w).  Batched cotangents -- torch.func.vmap over
the function returned by torch.func.vjp -- reach the multi-cotangent kernel
in one launch through the vmap rule of the inner adjoint Function.
"""

from __future__ import annotations

import torch


class _Adjoint(torch.autograd.Function):
    """(gx, gp) = adjoint of the residual at (x, params) for cotangent w."""

    @staticmethod
    def forward(x, params, w, plan):
        plan.set_params(params)
        gx, gp = plan.vjp(x, w.reshape(-1, 1).contiguous())
        return gx.reshape(-1), gp.reshape(-1)

    @staticmethod
    def setup_context(ctx, inputs, output):
        pass

    @staticmethod
    def vmap(info, in_dims, x, params, w, plan):
        if in_dims[0] is not None or in_dims[1] is not None:
            raise NotImplementedError("the adjoint batches over cotangents only")
        wd = in_dims[2]
        if wd is None:
            gx, gp = _Adjoint.apply(x, params, w, plan)
            return (gx, gp), (None, None)
        W = w.movedim(wd, -1).contiguous()          # (n, k): cotangent-fastest
        plan.set_params(params)
        gx, gp = plan.vjp(x, W)
        return (gx, gp), (1, 1)


class PFResidual(torch.autograd.Function):
    @staticmethod
    def forward(x, params, plan):
        plan.set_params(params)
        return plan.eval_residual(x)

    @staticmethod
    def setup_context(ctx, inputs, output):
        x, params, plan = inputs
        ctx.save_for_backward(x, params)
        ctx.plan = plan

    @staticmethod
    def backward(ctx, gF):
        x, params = ctx.saved_tensors
        gx, gp = _Adjoint.apply(x, params, gF, ctx.plan)
        return gx, gp, None


def residual(x, params, plan):
    """Functional form of PFResidual.apply."""
    return PFResidual.apply(x, params, plan)
