"""Differentiable Gabor feature layer: libgabor's forward bank and its
hand-written adjoint behind ``torch.autograd.Function``.

The forward is ``gabor_bank_apply`` (``gabor_bank_apply_batched`` for a
batch); the backward is ``gabor_bank_apply_adjoint`` (``..._batched``),
which maps dL/dF (complex64, PyTorch's convention dL/dRe F + i dL/dIm F) to
dL/df.  Both run in libgabor's HIP kernels; nothing here computes.
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
    """F[b] = bank(f[b]) for a float32 [B, H, W] batch into one complex64
    [B, O, N, H, W] output (one batched forward call); the backward is one
    batched adjoint call into a [B, H, W] gradient."""

    @staticmethod
    def forward(ctx, x, bank):
        ctx.bank = bank
        return bank.apply_batched(x.contiguous())

    @staticmethod
    def backward(ctx, grad_out):
        return ctx.bank.adjoint_batched(grad_out.contiguous()), None


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
