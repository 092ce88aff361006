"""Differentiable Gabor feature layer: libgabor's forward bank and its
hand-written adjoint behind ``torch.autograd.Function``.

The forward is ``gabor_bank_apply``; the backward is
``gabor_bank_apply_adjoint``, which maps dL/dF (complex64, PyTorch's
convention dL/dRe F + i dL/dIm F) to dL/df.  Both run in libgabor's HIP
kernels; nothing here computes.  The adjoint exists for the zero boundary
only, so the layer always plans with it.
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


class GaborLayer(torch.nn.Module):
    """Gabor bank over a batch of single-channel images.

    ``layer(x)`` takes float32 [B, H, W] (or [H, W]) on the GPU and returns
    complex64 [B, O, N, H, W] (or [O, N, H, W]).  The bank has no trainable
    parameters; gradients flow to the input.  One plan serves every image,
    so calls on the layer must not overlap across streams.
    """

    def __init__(self, height, width, omegas, sigmas, n_orient=None, thetas=None, radius_sigmas=3.0,
                 precision="fp32"):
        super().__init__()
        self.bank = binding.GaborBank(height, width, omegas, sigmas, n_orient, thetas, radius_sigmas,
                                      "zero", precision)

    def forward(self, x):
        if x.dim() == 2:
            return GaborBankFunction.apply(x, self.bank)
        if x.dim() != 3:
            raise ValueError("expected [B, H, W] or [H, W]")
        return torch.stack([GaborBankFunction.apply(x[b], self.bank) for b in range(x.shape[0])])

    def close(self):
        self.bank.close()
