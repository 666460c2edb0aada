"""The smoothed objective as a torch.autograd.Function.

forward(theta) = Q-hat, the mean per-image loss over N perturbed renders with
Gaussian perturbations tau ~ kappa (Sec. 3.1, Eq. 6-7 read with the kernel as
the sampling density), computed by the HIP library in one stream-ordered call.
backward(grad_out) = grad_out * g-hat, where g-hat is the plateau-reduced
gradient (Sec. 3.1, Eq. 10 with antithetic pairs), recombined on the device by
the library's binary64 combine kernel from the per-image losses and pair
weights saved by forward.  Torch supplies only memory and the stream.
"""
from __future__ import annotations

import torch

from . import native as NV


class PrdptSmoothedLoss(torch.autograd.Function):
    """Q-hat(theta) with the plateau-reduced gradient as its backward.

    Arguments: theta (device float32 tensor [d], the parameters), scene
    (native.Scene), ref (device float32 [H, W, 3]), sigma (device float32 [d]
    or a sequence), N (even number of renders), seed, est (estimator mode for
    the perturbations; GAUSS makes forward and backward the value and gradient
    of the same Monte Carlo estimate of Q).
    """

    @staticmethod
    def forward(ctx, theta, scene, ref, sigma, N, seed, est=NV.PRDPT_EST_GAUSS):
        dev = theta.device
        if not isinstance(sigma, torch.Tensor):
            sigma = torch.tensor(sigma, dtype=torch.float32, device=dev)
        sigma = sigma.to(device=dev, dtype=torch.float32).contiguous()
        th = theta.detach().to(torch.float32).contiguous()
        d = scene.d
        rows = N if int(est) & NV.PRDPT_EST_INDEPENDENT else N // 2   # weight rows
        if th.numel() != d or sigma.numel() != d:
            raise ValueError("theta/sigma length must equal the scene's parameter count")
        stream = torch.cuda.current_stream(dev)
        if stream.cuda_stream != getattr(scene.ctx.stream, "cuda_stream", None):
            scene.ctx.set_stream(stream)
        grad = torch.empty(d, dtype=torch.float64, device=dev)
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        losses = torch.empty(N, dtype=torch.float64, device=dev)
        c = torch.empty(rows, d, dtype=torch.float64, device=dev)
        NV.prdpt_grad_estimate_async(scene, ref.contiguous(), th, sigma, N, seed, est, grad, loss,
                                     losses, c)
        ctx.save_for_backward(losses, c)
        ctx.scene = scene
        ctx.est = int(est)
        ctx.theta_dtype = theta.dtype
        return loss[0].to(theta.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        losses, c = ctx.saved_tensors
        rows, d = c.shape
        scale = grad_out.detach().reshape(1).to(torch.float64).contiguous()
        g = torch.empty(d, dtype=torch.float64, device=c.device)
        NV.prdpt_combine_async(ctx.scene.ctx, rows, d, c, losses, scale, g, ctx.est)
        return g.to(ctx.theta_dtype), None, None, None, None, None, None


def smoothed_loss(theta, scene, ref, sigma, N, seed, est=NV.PRDPT_EST_GAUSS):
    """Functional form of PrdptSmoothedLoss.apply."""
    return PrdptSmoothedLoss.apply(theta, scene, ref, sigma, N, seed, est)
