"""GPU parity over seeded random configurations: image shape, frequencies
and radii (every operand quarter of the fused kernel, R = 0 .. 104, and the
two-pass kernels beyond), orientation count, boundary rule and arithmetic
form, each compared with the FP64 oracle at every pixel.

Bar per channel: the larger of the fixed cases' peak-relative bar (1e-5 for
FP32 and the FP16 split, 1e-3 for the BF16 split) and the form's absolute
rounding bound 8 u max|f| (|F| <= max|f| because the taps' magnitudes sum to
one; four operand roundings over two passes; u = 2^-9, 2^-12 for single
BF16, FP16 products, 2^-16, 2^-22 for their hi/lo splits, 16 x 2^-24 for FP32
with its accumulation).  The second term matters only for channels whose
response nearly cancels, such as a vertical channel of a 3-row image under
the mirror rule, where the folded signal repeats every 4 rows."""
import math

import numpy as np
import pytest

import oracle
from paper_1704_05231_amd import workloads

pytestmark = pytest.mark.gpu

TOLS = {"fp32": 1e-5, "fp16_split": 1e-5, "bf16_split": 1e-3, "fp16": 0.0, "bf16": 0.0}
UNIT = {"bf16": 2.0 ** -9, "fp16": 2.0 ** -12, "bf16_split": 2.0 ** -16, "fp16_split": 2.0 ** -22,
        "fp32": 16 * 2.0 ** -24}
PRECISIONS = ["fp32", "fp16_split", "bf16_split", "fp16", "bf16"]


def draw(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    H = int(rng.integers(1, 90))
    W = int(rng.integers(1, 100))
    n_freq = int(rng.integers(1, 3))
    # radius R = floor(3 sigma + 1/2): cover small, medium and large bands
    radii = [int(rng.choice([0, 1, 3, 6, 10, 20, 27, 30, 40, 45, 56, 57, 70, 88, 104, 110]))
             for _ in range(n_freq)]
    sigmas = [max(r, 0.1) / 3.0 if r > 0 else 0.1 for r in radii]
    omegas = [float(rng.uniform(0.0, math.pi)) for _ in range(n_freq)]
    n_orient = int(rng.integers(1, 9))
    boundary = "mirror" if rng.integers(0, 2) else "zero"
    prec = PRECISIONS[int(rng.integers(0, len(PRECISIONS)))]
    return H, W, omegas, sigmas, n_orient, boundary, prec


@pytest.mark.parametrize("seed", range(96))
def test_random_configuration(gpu_lib, seed):
    import torch
    H, W, om, sg, N, bnd, prec = draw(700 + seed)
    img = workloads.uniform_image(H, W, 800 + seed)
    bank = gpu_lib.GaborBank(H, W, om, sg, N, None, 3.0, bnd, prec)
    got = bank(torch.from_numpy(img).cuda()).cpu().numpy()
    bank.close()
    ref = oracle.gabor_bank(img, om, sg, workloads.orientations(N), 3.0, bnd)
    num = np.abs(got - ref).reshape(len(om), N, -1).max(-1)
    peak = np.abs(ref).reshape(len(om), N, -1).max(-1)
    fmax = float(np.abs(img).max())
    bar = np.maximum(TOLS[prec] * peak, 8 * UNIT[prec] * fmax)
    radii = [int(math.floor(3 * s + 0.5)) for s in sg]
    print(f"seed {seed}: {H}x{W} N={N} R={radii} {bnd} {prec}: max err / peak "
          f"{(num / np.maximum(peak, 1e-300)).max():.3e}, max err / max|f| {num.max() / fmax:.3e}, "
          f"worst err / bar {(num / bar).max():.3f}")
    assert np.all(num <= bar)
