"""GPU parity of the recursive-smoother bank (gabor_bank_plan_iir) against
the oracle's FP64 implementation of the same recursion, and its quality as
an approximation of Eq. (1) (signal-to-error ratio against the direct sum).

Bar for FP32 against FP64 of the same recursion, per channel of frequency
i: peak-relative error <= max(1e-5, 8 u / a0(sigma_i)), u = 2^-24.  Rounding
errors of each step are amplified by the recursion's gain 1 / a0 (the DC
gain of the all-pole part), which grows like sigma^3 (a0 is about 4e-2 at
sigma = 4 and 9e-4 at sigma = 16); four recursions run in sequence
(forward and backward, both axes), and the factor 8 leaves a factor of two
for the modulation roundings.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1704_05231_amd import workloads

pytestmark = pytest.mark.gpu

def bar(sigmas):
    """Per-frequency bar, shape [O, 1] against errors [O, N]."""
    return np.array([[max(1e-5, 8 * 2.0 ** -24 / oracle.iir_coeffs(s)[0])] for s in sigmas])

CASES = [
    # (H, W, omegas, sigmas, n_orient, thetas, boundary)
    (37, 53, [math.pi / 4, 1.3], [2.0, 1.5], 8, None, "mirror"),
    (64, 80, [math.pi / 2, math.pi / 8], [2.0, 8.0], 8, None, "zero"),
    (9, 11, [0.9], [4.0], 5, None, "mirror"),            # lines shorter than the extension
    (1, 40, [1.0], [1.5], 3, None, "mirror"),            # one row
    (70, 129, [0.7, 0.0], [3.0, 0.8], 7, None, "zero"),  # odd N, omega = 0, small sigma
    (48, 40, [1.1], [2.2], 5, [0.0, 0.4, math.pi - 0.4, 1.0, math.pi / 2], "mirror"),
    (96, 110, [math.pi / 16], [16.0], 4, None, "mirror"),
    # rows beyond the register kernel's 4096 extended samples: the horizontal
    # pass keeps its forward results in the scratch plane (16 rows: with 3
    # the mirror-folded columns repeat every 4 rows and the sigma = 4
    # vertical channels cancel to 1 % of the input, where a peak-relative
    # bar measures the cancellation, not the recursion)
    (16, 4300, [1.0, math.pi / 4], [1.5, 4.0], 4, None, "mirror"),
    (2, 4200, [0.6], [2.0], 3, None, "zero"),
    # the horizontal pass writes its lines as rows through LDS in rounds of
    # whole waves: chunk lengths 16, 32, 40 and 48 (1024 columns: 24)
    (30, 700, [0.9], [2.0], 4, None, "mirror"),
    (20, 2000, [1.2, 0.5], [1.0, 3.0], 3, None, "zero"),
    (16, 2400, [1.0], [2.5], 2, None, "mirror"),
    (16, 2900, [0.8], [2.0], 4, None, "mirror"),
]


def gpu_iir(gpu_lib, img, om, sg, N, th, bnd):
    import torch
    bank = gpu_lib.GaborBank(img.shape[0], img.shape[1], om, sg, N, th, 3.0, bnd, "fp32", smoother="iir")
    out = bank(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    bank.close()
    return res


def rel_err(got, ref):
    num = np.abs(got - ref).reshape(*ref.shape[:2], -1).max(-1)
    den = np.abs(ref).reshape(*ref.shape[:2], -1).max(-1)
    return num / den


@pytest.mark.parametrize("case", range(len(CASES)))
def test_iir_matches_oracle_recursion(gpu_lib, case):
    H, W, om, sg, N, th, bnd = CASES[case]
    img = workloads.uniform_image(H, W, 900 + case)
    thetas = workloads.orientations(N) if th is None else np.asarray(th)
    got = gpu_iir(gpu_lib, img, om, sg, N, th, bnd)
    ref = oracle.gabor_bank_iir(img, om, sg, thetas, bnd)
    err = rel_err(got, ref)
    print(f"iir case {case} {H}x{W} {bnd}: max rel err {err.max():.3e}")
    assert np.all(err <= bar(sg))


def ser_db(gpu_lib, img, om, sg, N, bnd, n_pts, seed):
    got = gpu_iir(gpu_lib, img, om, sg, N, None, bnd)
    H, W = img.shape
    xs, ys = workloads.sample_pixels(H, W, n_pts, seed)
    ref = oracle.gabor_bank_points(img, om, sg, workloads.orientations(N), xs, ys, 5.0, bnd)
    g = got[:, :, ys, xs].transpose(2, 0, 1)
    return 10 * np.log10((np.abs(ref) ** 2).sum(0) / (np.abs(g - ref) ** 2).sum(0))


def test_iir_approximates_eq1(gpu_lib):
    """512^2 smoothed noise, 8 orientations, sigma = 2, 4, 8 with w sigma = 1
    (the recursive Gaussian's accurate range), mirror: SER of the recursive
    form against the direct sum with the Gaussian to 5 sigma, at sampled
    pixels, above 27 dB on every channel (about 34 dB measured on the CPU
    with the oracle's own recursion)."""
    img = workloads.smoothed_image(512, 512, 7)
    sg = [2.0, 4.0, 8.0]
    ser = ser_db(gpu_lib, img, [1 / s for s in sg], sg, 8, "mirror", 400, 905)
    print("SER dB per channel", np.round(ser, 1))
    assert ser.min() > 27.0


def test_iir_on_the_metric_bank(gpu_lib):
    """The metric workload's bank (sigma = pi / w: w sigma = pi, a one-octave
    Gabor): far from DC the third-order recursion's frequency response errs
    most, and the SER drops to about 10-15 dB on the axis orientations and
    about 28-33 dB on the diagonal ones (oracle recursion, CPU); reported,
    with a sanity bar only."""
    wl = workloads.bank_1024()
    img = workloads.smoothed_image(512, 512, 7)
    ser = ser_db(gpu_lib, img, wl.omegas, wl.sigmas, 8, "mirror", 400, 906)
    print("SER dB per channel", np.round(ser, 1))
    assert ser.min() > 5.0


def test_iir_plan_has_no_adjoint_or_batch(gpu_lib):
    import torch
    bank = gpu_lib.GaborBank(16, 16, [1.0], [2.0], 4, None, 3.0, "zero", "fp32", smoother="iir")
    with pytest.raises(gpu_lib.GaborError) as ei:
        bank.adjoint(torch.zeros((1, 4, 16, 16), dtype=torch.complex64, device="cuda"))
    assert ei.value.status == 4
    with pytest.raises(gpu_lib.GaborError) as ei:
        gpu_lib.GaborBatch(bank, [torch.zeros((16, 16), device="cuda")])
    assert ei.value.status == 4
    bank.close()


def draw(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W = int(rng.integers(1, 90)), int(rng.integers(1, 130))
    n_freq = int(rng.integers(1, 3))
    sigmas = [float(rng.uniform(0.5, 12.0)) for _ in range(n_freq)]
    omegas = [float(rng.uniform(0.0, math.pi)) for _ in range(n_freq)]
    boundary = "mirror" if rng.integers(0, 2) else "zero"
    return H, W, omegas, sigmas, int(rng.integers(1, 9)), boundary


@pytest.mark.parametrize("seed", range(24))
def test_iir_random_configuration(gpu_lib, seed):
    """Seeded random shapes (1..89 x 1..129), sigma in [0.5, 12], frequencies,
    orientation counts and rules against the oracle's FP64 recursion."""
    H, W, om, sg, N, bnd = draw(950 + seed)
    img = workloads.uniform_image(H, W, 970 + seed)
    got = gpu_iir(gpu_lib, img, om, sg, N, None, bnd)
    ref = oracle.gabor_bank_iir(img, om, sg, workloads.orientations(N), bnd)
    err = rel_err(got, ref)
    print(f"iir seed {seed} {H}x{W} sigma {sg} N={N} {bnd}: max rel err {err.max():.3e}, "
          f"worst err / bar {(err / bar(sg)).max():.3f}")
    assert np.all(err <= bar(sg))
