"""GPU parity: libgabor through its C ABI against the FP64 oracle.

Error measure (per channel): max over pixels of |F_gpu - F_ref| divided by
max over pixels of |F_ref| ("relative to the peak response"), held to the
form's bar of tests/bars.py: 1e-5 for FP32 and the float16 split, 1e-3 for
the bfloat16 split, 4e-3 and 4e-2 for single float16 and bfloat16
products.
"""
import math

import numpy as np
import pytest

import oracle
from bars import channel_bars
from paper_1704_05231_amd import workloads

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
PRECISIONS = ["fp32", "fp16_split", "bf16_split", "fp16", "bf16"]


def check(prec, img, got, ref):
    """Per-channel errors of arrays [..., H, W] against the form's bars
    (tests/bars.py): the worst ratio error / bar, which must be <= 1."""
    num = np.abs(got - ref).reshape(*ref.shape[:-2], -1).max(-1)
    peak = np.abs(ref).reshape(*ref.shape[:-2], -1).max(-1)
    bar, n_cancel = channel_bars(prec, float(np.abs(img).max()), peak)
    ratio = num / np.maximum(bar, 1e-300)
    return ratio, n_cancel


def gpu_bank(binding, img, omegas, sigmas, n_orient, thetas=None, boundary="zero",
             precision="fp32", radius_sigmas=3.0, stride_pad=0):
    import torch
    H, W = img.shape
    buf = torch.zeros((H, W + stride_pad), dtype=torch.float32, device="cuda")
    buf[:, :W] = torch.from_numpy(img).cuda()
    view = buf[:, :W]
    bank = binding.GaborBank(H, W, omegas, sigmas, n_orient, thetas, radius_sigmas, boundary,
                             precision)
    out = bank(view)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    bank.close()
    return res


def rel_err(got, ref):
    """Per-channel peak-relative error, arrays [..., H, W] -> [...]."""
    num = np.abs(got - ref).reshape(*ref.shape[:-2], -1).max(-1)
    den = np.abs(ref).reshape(*ref.shape[:-2], -1).max(-1)
    return num / np.maximum(den, 1e-300)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_bank_small_full_grid(gpu_lib, prec):
    wl = workloads.bank_small()
    img = wl.images[0]
    got = gpu_bank(gpu_lib, img, wl.omegas, wl.sigmas, wl.n_orient, wl.thetas, wl.boundary, prec)
    ref = oracle.gabor_bank(img, wl.omegas, wl.sigmas, wl.thetas, 3.0, wl.boundary)
    err = rel_err(got, ref)
    ratio, nc = check(prec, img, got, ref)
    print(f"bank-256 {prec} per-channel rel err max {err.max():.3e}, worst err/bar {ratio.max():.3f}, "
          f"{nc} cancelling channels")
    assert np.all(ratio <= 1)


CASES = [
    # (H, W, omegas, sigmas, n_orient, thetas, boundary)
    (37, 53, [math.pi / 4, 1.3], [2.0, 1.5], 8, None, "mirror"),
    (64, 63, [math.pi / 2, math.pi / 8], [2.0, 8.0], 8, None, "zero"),
    (9, 11, [0.9], [4.0], 5, None, "mirror"),           # R = 12 > both sides
    (9, 11, [0.9], [4.0], 5, None, "zero"),
    (1, 17, [1.0], [1.5], 3, None, "mirror"),          # one row
    (23, 1, [1.0], [1.5], 4, None, "mirror"),          # one column
    (1, 1, [2.0], [1.0], 2, None, "zero"),
    (70, 129, [0.7, 2.1, 0.0], [3.0, 1.0, 2.0], 7, None, "zero"),     # odd N, omega = 0
    (48, 40, [1.1], [2.2], 5, [0.0, 0.4, math.pi - 0.4, 1.0, math.pi / 2], "mirror"),  # unpaired 1.0
    (33, 65, [0.8], [1.7], 4, [math.pi / 2, 3 * math.pi / 2, -0.3, math.pi + 0.3], "zero"),
    (130, 300, [math.pi / 16], [16.0], 8, None, "mirror"),             # R = 48 over a ragged tile
    (150, 170, [math.pi / 30, 0.2], [25.0, 12.0], 6, None, "mirror"),  # R = 75, 36
    (90, 200, [math.pi / 32], [32.0], 4, None, "zero"),               # R = 96 > image height
]


@pytest.mark.parametrize("prec", PRECISIONS + ["fp32_twopass"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_bank_shapes_full_grid(gpu_lib, case, prec, monkeypatch):
    H, W, om, sg, N, th, bnd = CASES[case]
    if prec == "fp32_twopass":
        monkeypatch.setenv("LIBGABOR_ALGO", "twopass")
        prec = "fp32"
    img = workloads.uniform_image(H, W, 100 + case)
    thetas = workloads.orientations(N) if th is None else np.asarray(th)
    got = gpu_bank(gpu_lib, img, om, sg, N, th, bnd, prec)
    ref = oracle.gabor_bank(img, om, sg, thetas, 3.0, bnd)
    err = rel_err(got, ref)
    ratio, nc = check(prec, img, got, ref)
    print(f"case {case} {H}x{W} N={N} {bnd} {prec}: max rel err {err.max():.3e}, worst err/bar "
          f"{ratio.max():.3f}, {nc} cancelling channels")
    assert np.all(ratio <= 1)


def test_row_stride_larger_than_width(gpu_lib):
    img = workloads.uniform_image(40, 50, 7)
    om, sg = [0.6, 1.4], [2.5, 1.2]
    a = gpu_bank(gpu_lib, img, om, sg, 6, boundary="mirror")
    b = gpu_bank(gpu_lib, img, om, sg, 6, boundary="mirror", stride_pad=13)
    np.testing.assert_array_equal(a, b)


def test_repeat_runs_are_bitwise_identical(gpu_lib):
    import torch
    wl = workloads.bank_small()
    bank = gpu_lib.GaborBank(256, 256, wl.omegas, wl.sigmas, 4, wl.thetas, 3.0, "zero")
    img = torch.from_numpy(wl.images[0]).cuda()
    a = bank(img).cpu()
    b = bank(img).cpu()
    bank.close()
    assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))


@pytest.fixture(scope="module")
def bank_1024_ref():
    wl = workloads.bank_1024()
    xs, ys = workloads.sample_pixels(1024, 1024, 2000, 42)
    ref = oracle.gabor_bank_points(wl.images[0], wl.omegas, wl.sigmas, wl.thetas_or_default,
                                   xs, ys, 3.0, wl.boundary)            # [P, O, N]
    return wl, xs, ys, ref


@pytest.mark.parametrize("prec", PRECISIONS)
def test_bank_1024_sampled(gpu_lib, bank_1024_ref, prec):
    """Full metric workload (1024^2, 8 x 4 bank, mirror) in the benchmark's
    launch configuration, checked at sampled pixels (corners included)."""
    wl, xs, ys, ref = bank_1024_ref
    img = wl.images[0]
    got = gpu_bank(gpu_lib, img, wl.omegas, wl.sigmas, wl.n_orient, None, wl.boundary, prec)
    g = got[:, :, ys, xs].transpose(2, 0, 1)
    peak = np.abs(ref).max(0)          # oracle peak over the samples (<= true peak: stricter)
    err = (np.abs(g - ref).max(0) / peak)
    bar, nc = channel_bars(prec, float(np.abs(img).max()), peak)
    ratio = np.abs(g - ref).max(0) / bar
    print(f"bank-1024 {prec} sampled max rel err {err.max():.3e}, worst err/bar {ratio.max():.3f}, "
          f"{nc} cancelling channels")
    assert nc == 0 and np.all(ratio <= 1)
