"""torch.autograd.Function around the C ABI: forward = ciq_invsqrt_mvm or
ciq_sqrt_mvm (keeping the per-shift solves), backward = ciq_backward
(gradients for B, lengthscale(s), outputscale and noise)."""
from __future__ import annotations

import numpy as np
import torch

from . import ops


class CIQFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, x, lengthscale, outputscale, noise, kernel, mode, q, max_iter, tol, bounds, precision):
        ls = lengthscale.detach().double().cpu().numpy().reshape(-1)
        prob = ops.Problem(x.detach(), kernel, ls, float(outputscale), float(noise))
        fn = ops.ciq_sqrt_mvm if mode == "sqrt" else ops.ciq_invsqrt_mvm
        out, info, solves = fn(prob, b.detach(), q=q, max_iter=max_iter, tol=tol, bounds=bounds,
                               precision=precision, keep_solves=True)
        ctx.save_for_backward(x, solves, lengthscale, outputscale, noise)
        ctx.meta = (kernel, mode, max_iter, tol, precision, info["t"], info["w"], ls)
        ctx.info = info
        return out

    @staticmethod
    def backward(ctx, grad_out):
        x, solves, lengthscale, outputscale, noise = ctx.saved_tensors
        kernel, mode, max_iter, tol, precision, t, w, ls = ctx.meta
        prob = ops.Problem(x.detach(), kernel, ls, float(outputscale), float(noise))
        need_b = ctx.needs_input_grad[0]
        need_h = any(ctx.needs_input_grad[2:5])
        db, dls, do2, dn, _ = ops.ciq_backward(prob, grad_out.contiguous(), t, w, solves, mode=mode,
                                               max_iter=max_iter, tol=tol, precision=precision,
                                               want_b=need_b, want_hyper=need_h)

        def like(v, ref):
            return torch.as_tensor(np.asarray(v), dtype=ref.dtype, device=ref.device).reshape(ref.shape)

        g_ls = like(dls, lengthscale) if need_h and ctx.needs_input_grad[2] else None
        g_o2 = like(do2, outputscale) if need_h and ctx.needs_input_grad[3] else None
        g_s2 = like(dn, noise) if need_h and ctx.needs_input_grad[4] else None
        return db, None, g_ls, g_o2, g_s2, None, None, None, None, None, None, None


def ciq_apply(b, x, lengthscale, outputscale, noise, kernel="rbf", mode="invsqrt", q=15, max_iter=200,
              tol=1e-4, bounds=None, precision=None):
    """Differentiable K^{-1/2} b (mode 'invsqrt') or K^{1/2} b (mode 'sqrt')."""
    return CIQFunction.apply(b, x, lengthscale, outputscale, noise, kernel, mode, q, max_iter, tol, bounds,
                             precision)
