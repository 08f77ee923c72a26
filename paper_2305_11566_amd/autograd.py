"""torch.autograd.Function over the hand-written forward and backward kernels.

    out, mu_logvar = SvRefine.apply(params, refiner, disp_low, img_low, H, W, eps)

params is the FP32 canonical parameter vector (requires_grad); it is packed
into the refiner's compute dtype on every call.  Any torch loss on out and
mu_logvar can follow; backward calls sv_vae_backward with the incoming
gradients (the KL weight of the library call is 0: a KL written in torch on
mu_logvar reaches the kernels as the mu/logvar gradient).
"""
from __future__ import annotations

import torch


class SvRefine(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, refiner, disp_low, img_low, H, W, eps=None):
        refiner.pack(params.detach().contiguous())
        B = disp_low.shape[0]
        saved = refiner.saved_buffer(B, H, W)
        out, ml = refiner.forward(disp_low, img_low, H, W, eps=eps, saved=saved)
        ctx.refiner, ctx.saved, ctx.eps, ctx.shape = refiner, saved, eps, (B, H, W)
        return out, ml

    @staticmethod
    def backward(ctx, dout, dml):
        B, H, W = ctx.shape
        if dout is None:
            dout = torch.zeros((B, H, W), dtype=torch.float32, device=ctx.saved.device)
        g = ctx.refiner.backward(ctx.saved, B, H, W, ctx.eps, dout.contiguous().float(), 0.0,
                                 dmu_logvar=None if dml is None else dml.contiguous().float())
        return g, None, None, None, None, None, None
