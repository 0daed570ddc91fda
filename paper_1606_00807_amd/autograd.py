"""torch.autograd.Function over fit + analysis.

X_a = EnKF-MC analysis of X_b (eq. 1 / eq. 8 fit with ridge lam, eq. 11 local
solves, merge of Alg. 2).  The backward pass is the library's hand-written
adjoint (enkfmc_analyze_backward): it recomputes each regression's Gram and
Cholesky factor instead of storing them, and returns dL/dX_b, dL/dlog r and
dL/dlam.  When the plan has been used since (another cycle of a chain), the
backward pass first recomputes this call's fit and analysis on the saved
inputs, so a chain of analyses on one plan keeps only its inputs alive.
"""
from __future__ import annotations

import torch

from .api import Plan


class EnkfmcAnalysis(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Xb, log_r, ridge, plan: Plan, Y, mode: str = "batched"):
        lam = float(ridge.detach().cpu()) if isinstance(ridge, torch.Tensor) else float(ridge)
        Xd = Xb.detach()
        plan.fit(Xd, lam, mode=mode)
        r = torch.exp(log_r.detach().to(torch.float64))
        Xa = plan.analyze(Xd, Y, r)
        ctx.plan = plan
        ctx.token = plan.analysis_token
        ctx.inputs = (r, lam, mode)
        # Y (the device copy the analysis read, possibly the caller's own
        # tensor) goes through save_for_backward, so that overwriting it in
        # place before the reverse pass raises instead of giving wrong
        # gradients
        ctx.save_for_backward(Xd, plan._analysis_inputs[0])
        ctx.meta = (Xb.dtype, log_r.dtype, ridge.dtype if isinstance(ridge, torch.Tensor) else None,
                    ridge.shape if isinstance(ridge, torch.Tensor) else None)
        return Xa

    @staticmethod
    def backward(ctx, gXa):
        Xd, Yd = ctx.saved_tensors
        plan = ctx.plan
        if plan.analysis_token != ctx.token:
            r, lam, mode = ctx.inputs
            plan.fit(Xd, lam, mode=mode)
            plan.analyze(Xd, Yd, r)
        dXb, dlogR, dridge = plan.backward(Xd, gXa.detach())
        xdt, rdt, ldt, lshape = ctx.meta
        gl = dridge.to(ldt).reshape(lshape) if ldt is not None else None
        return dXb.to(xdt), dlogR.to(rdt), gl, None, None, None


def enkfmc_analysis(Xb, log_r, ridge, plan: Plan, Y, mode: str = "batched"):
    """Differentiable X_a(X_b, log r, lam) on one plan (one GPU)."""
    return EnkfmcAnalysis.apply(Xb, log_r, ridge, plan, Y, mode)
