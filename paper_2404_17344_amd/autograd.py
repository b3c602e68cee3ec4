"""torch.autograd.Function for y = K(l, sigma) v with a hand-written backward.

Backward returns
  dL/dv       = K g                       (K is symmetric)
  dL/dl_w     = <g, sigma_w^2 dK_w/dl_w v>
  dL/dsigma_w = <g, 2 sigma_w K_w v>
computed by ``addk_vjp``: the scalar gradients are Fourier-domain inner
products of the transformed v and g with the kernel and derivative-kernel
multipliers, i.e. exact derivatives of the approximate operator with the torus
period held fixed (derivatives of the section "Implementing the NFFT approach").

The plan holds one set of parameters.  Forward sets the plan to the call's
(l, sigma) and records them; backward evaluates at the recorded values, so a
graph stays correct when other forwards at other parameters ran in between,
and puts the plan's parameters back afterwards.
"""
from __future__ import annotations

import numpy as np
import torch


def _set_params(plan, ell_h, sig_h):
    if not (np.array_equal(ell_h, plan.ell) and np.array_equal(sig_h, plan.sigma)):
        plan.update_params(ell_h, sig_h)


class KernelMatvec(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, ell, sigma, plan):
        ell_h = ell.detach().cpu().numpy().astype(np.float64)
        sig_h = sigma.detach().cpu().numpy().astype(np.float64)
        _set_params(plan, ell_h, sig_h)
        ctx.plan = plan
        ctx.params = (ell_h, sig_h)
        ctx.vdim = V.dim()
        ctx.save_for_backward(V)
        Y = plan.matvec(V)
        return Y[:, 0] if V.dim() == 1 else Y

    @staticmethod
    def backward(ctx, G):
        (V,) = ctx.saved_tensors
        plan = ctx.plan
        need_v, need_l, need_s = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        before = (plan.ell.copy(), plan.sigma.copy())
        _set_params(plan, *ctx.params)
        try:
            gV, gl, gs = plan.vjp(V, G.contiguous(), want_v=need_v, want_params=need_l or need_s)
        finally:
            _set_params(plan, *before)
        if gV is not None and ctx.vdim == 1:
            gV = gV[:, 0]
        return gV, (gl if need_l else None), (gs if need_s else None), None
