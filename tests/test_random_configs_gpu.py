"""GPU parity over seeded random configurations: image shape, frequencies
and radii (every operand quarter of the fused kernel, R = 0 .. 104, and the
two-pass kernels beyond), orientation count, boundary rule and arithmetic
form, each compared with the FP64 oracle at every pixel.

Bar per channel: the form's peak-relative bar of tests/bars.py (1e-5 for
FP32 and the float16 split, 1e-3 for the bfloat16 split, 4e-3 and 4e-2 for
single float16 and bfloat16 products); only channels whose response nearly
cancels (peak below 1e-2 of max|f|, such as a vertical channel of a 3-row
mirror-extended image, whose folded signal repeats every 4 rows) take the
form's absolute rounding bound 8 u max|f| instead, and their count is
printed."""
import math

import numpy as np
import pytest

import oracle
from bars import channel_bars
from paper_1704_05231_amd import workloads

pytestmark = pytest.mark.gpu

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
    bar, nc = channel_bars(prec, fmax, peak)
    radii = [int(math.floor(3 * s + 0.5)) for s in sg]
    print(f"seed {seed}: {H}x{W} N={N} R={radii} {bnd} {prec}: max err / peak "
          f"{(num / np.maximum(peak, 1e-300)).max():.3e}, max err / max|f| {num.max() / fmax:.3e}, "
          f"worst err / bar {(num / bar).max():.3f}, {nc} of {num.size} channels cancelling")
    assert np.all(num <= bar)
