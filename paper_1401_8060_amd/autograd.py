"""torch.autograd binding of the smooth statistic.

The forward pass calls the library's forward kernel (stt_smooth); the
backward pass calls its hand-written gradient kernel (stt_grad) and scales the
result by the incoming gradient. Nothing is differentiated by torch itself.
"""
from __future__ import annotations

import torch


class SmoothSNR(torch.autograd.Function):
    """z~(theta) per template: theta [n][6] float32 (tau0, tau2, phi0, phi1, phi2, dtau_ms), K [n] int32."""

    @staticmethod
    def forward(fctx, theta, K, ctx, m):
        theta_c = theta.detach().contiguous()
        fctx.save_for_backward(theta_c, K)
        fctx.stt = (ctx, m)
        return ctx.smooth(m, theta_c, K)

    @staticmethod
    def backward(fctx, gz):
        theta_c, K = fctx.saved_tensors
        ctx, m = fctx.stt
        _, g = ctx.grad(m, theta_c, K)
        return gz.to(g.dtype)[:, None] * g, None, None, None


def smooth_snr(ctx, m, theta: torch.Tensor, K: torch.Tensor) -> torch.Tensor:
    return SmoothSNR.apply(theta, K, ctx, m)
