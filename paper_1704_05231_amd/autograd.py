"""Differentiable Gabor feature layer: libgabor's forward bank and its
hand-written adjoint behind ``torch.autograd.Function``.

The forward is ``gabor_bank_apply``; the backward is
``gabor_bank_apply_adjoint``, which maps dL/dF (complex64, PyTorch's
convention dL/dRe F + i dL/dIm F) to dL/df.  Both run in libgabor's HIP
kernels; nothing here computes.  The mirror rule's adjoint needs every
frequency in the fused kernel (R <= 56); the zero boundary has no limit.
"""
from __future__ import annotations

import torch

from . import binding


class GaborBankFunction(torch.autograd.Function):
    """F = bank(f) for one (H, W) float32 image; backward through the adjoint."""

    @staticmethod
    def forward(ctx, img, bank):
        ctx.bank = bank
        return bank(img.contiguous())

    @staticmethod
    def backward(ctx, grad_out):
        grad_img = ctx.bank.adjoint(grad_out.contiguous())
        return grad_img, None


class GaborBatchFunction(torch.autograd.Function):
    """F[b] = bank(f[b]) for a float32 [B, H, W] batch, every image written
    straight into its slice of one complex64 [B, O, N, H, W] output; the
    backward writes each image's dL/df into its slice of one [B, H, W]
    gradient."""

    @staticmethod
    def forward(ctx, x, bank):
        ctx.bank = bank
        x = x.contiguous()
        out = torch.empty((x.shape[0], bank.n_freq, bank.n_orient, bank.height, bank.width),
                          dtype=torch.complex64, device=x.device)
        for b in range(x.shape[0]):
            bank(x[b], out[b])
        return out

    @staticmethod
    def backward(ctx, grad_out):
        grad_out = grad_out.contiguous()
        bank = ctx.bank
        grad = torch.empty((grad_out.shape[0], bank.height, bank.width), dtype=torch.float32,
                           device=grad_out.device)
        for b in range(grad_out.shape[0]):
            bank.adjoint(grad_out[b], grad[b])
        return grad, None


class GaborLayer(torch.nn.Module):
    """Gabor bank over a batch of single-channel images.

    ``layer(x)`` takes float32 [B, H, W] (or [H, W]) on the GPU and returns
    complex64 [B, O, N, H, W] (or [O, N, H, W]).  The bank has no trainable
    parameters; gradients flow to the input.  One plan serves every image,
    so calls on the layer must not overlap across streams.
    """

    def __init__(self, height, width, omegas, sigmas, n_orient=None, thetas=None, radius_sigmas=3.0,
                 precision="fp32", boundary="zero"):
        super().__init__()
        self.bank = binding.GaborBank(height, width, omegas, sigmas, n_orient, thetas, radius_sigmas,
                                      boundary, precision)

    def forward(self, x):
        if x.dim() == 2:
            return GaborBankFunction.apply(x, self.bank)
        if x.dim() != 3:
            raise ValueError("expected [B, H, W] or [H, W]")
        return GaborBatchFunction.apply(x, self.bank)

    def close(self):
        self.bank.close()
