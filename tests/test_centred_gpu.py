"""GPU checks of the local offset of the single 16-bit forms (BF16, FP16)
and of the FP32 form above R = 56: each workgroup subtracts a constant c from the image
before the passes and adds back c times the response to a constant, which
under the mirror rule is the same at every pixel:
    c (sum of the vertical taps)(sum of the horizontal taps)
(conjugated on the horizontal factor for the pi - theta partner).

Pin: a constant image whose value has few significant bits cancels to zero
before any rounding, so these forms must return the oracle's
response to a constant (Eq. (1) summed directly, the closed form
c A(w cos t) A(w sin t)) to FP32 accuracy, where without the offset they
would miss it by the 16-bit rounding of the image and the taps (about 1e-3
for FP16, 1e-2 for BF16).  This catches a wrong sign, conjugate or factor in
the correction for every job kind (theta = 0: real vertical taps; pi/2: real
J; the pairs).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1704_05231_amd import workloads

pytestmark = pytest.mark.gpu


# the single 16-bit forms use the offset at every radius, FP32 above R = 56
CONFIGS = {
    "bf16": ([math.pi / 2, math.pi / 8, 0.3], [2.0, 4.0, 3.0]),
    "fp16": ([math.pi / 2, math.pi / 8, 0.3], [2.0, 4.0, 3.0]),
    "fp32": ([math.pi / 20, 0.1], [20.0, 25.0]),                 # R = 60, 75
}


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_constant_image_is_exact_with_the_offset(gpu_lib, prec):
    import torch
    H, W = 70, 90
    c = 0.625
    img = np.full((H, W), c, dtype=np.float32)
    om, sg = CONFIGS[prec]
    th = workloads.orientations(8)
    bank = gpu_lib.GaborBank(H, W, om, sg, 8, None, 3.0, "mirror", prec)
    got = bank(torch.from_numpy(img).cuda()).cpu().numpy()
    bank.close()
    ref = oracle.gabor_bank(img, om, sg, th, 3.0, "mirror")
    peak = np.abs(ref).reshape(len(om), 8, -1).max(-1)
    err = np.abs(got - ref).reshape(len(om), 8, -1).max(-1) / peak
    print(prec, "constant image: per-channel peak-relative error max", err.max())
    assert err.max() < 2e-5
