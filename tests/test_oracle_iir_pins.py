"""Pins of the oracle's recursive-smoother variant (oracle.gabor_bank_iir):
what the recursion and the paper's modulate / smooth / demodulate order fix,
independently of the variant's own code path.

- The forward-then-backward recursion has an even impulse response with unit
  sum whose variance approximates sigma^2 (the design target of the
  recursive Gaussian).
- The modulated form reproduces the Gabor impulse response of Eq. (1) with
  the recursion's impulse response h in place of S:
      F(x, y) = h(x - x0) h(y - y0) exp(i w ((x - x0) cos t + (y - y0) sin t)).
- Linearity and the real-input symmetry F_(t + pi) = conj(F_t).
- The approximation of the direct Eq. (1) sum (Gaussian to 5 sigma) has a
  signal-to-error ratio near 30 dB (bar 27 dB).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1704_05231_amd import workloads


def impulse(H, W, y0, x0):
    img = np.zeros((H, W), dtype=np.float32)
    img[y0, x0] = 1.0
    return img


def line_response(sigma, n=None):
    """h(t), t = -c..c, from the oracle with w = 0 on an impulse."""
    c = int(math.ceil(16 * sigma)) + 20
    n = n or 2 * c + 1
    F = oracle.gabor_bank_iir(impulse(n, n, c, c), [0.0], [sigma], [0.0], "zero")[0, 0]
    h = F[c, :].real / F[c, c].real * F[c, c].real       # row through the centre
    hy = F[:, c].real
    # F(c, x) = h(0) h(x - c): divide by h(0) = sqrt(F(c, c))
    h0 = math.sqrt(F[c, c].real)
    return h / h0, hy / h0, F, c


@pytest.mark.parametrize("sigma", [1.0, 2.0, 4.0, 9.0])
def test_impulse_response_is_an_even_unit_sum_gaussian_approximation(sigma):
    h, hy, F, c = line_response(sigma)
    t = np.arange(-c, c + 1)
    np.testing.assert_allclose(h, h[::-1], rtol=0, atol=1e-10 * h.max())       # even
    np.testing.assert_allclose(h, hy, rtol=0, atol=1e-10 * h.max())            # same on both axes
    assert abs(h.sum() - 1.0) < 1e-6
    var = float((t ** 2 * h).sum())
    assert abs(var / sigma ** 2 - 1.0) < 0.05, var
    # the 2-D response is separable: F = h(y) h(x)
    np.testing.assert_allclose(F.real, np.outer(h, h), rtol=0, atol=1e-10 * F.real.max())
    g = np.exp(-t ** 2 / (2 * sigma ** 2))
    g /= g.sum()
    # the L2-optimal third-order design stays within a few per cent of the
    # sampled Gaussian's peak (worst at small sigma)
    assert np.abs(h - g).max() < 0.04 * g.max()


@pytest.mark.parametrize("theta", [0.0, 0.4, math.pi / 2, 2.5])
def test_modulated_impulse_is_the_gabor_kernel_with_h(theta):
    sigma, om = 3.0, 0.9
    h, _, _, c = line_response(sigma)
    n = 2 * c + 1
    F = oracle.gabor_bank_iir(impulse(n, n, c, c), [om], [sigma], [theta], "zero")[0, 0]
    t = np.arange(-c, c + 1)
    dx, dy = np.meshgrid(t, t)
    want = np.outer(h, h) * np.exp(1j * om * (dx * math.cos(theta) + dy * math.sin(theta)))
    assert np.abs(F - want).max() < 1e-10 * np.abs(want).max()


def test_linearity_and_conjugate_symmetry():
    # dyadic pixel values, so that 2a - 3b is exact in FP32
    a = np.round(workloads.uniform_image(30, 41, 61) * 256).astype(np.float32) / 256
    b = np.round(workloads.uniform_image(30, 41, 62) * 256).astype(np.float32) / 256
    om, sg = [0.8, 0.3], [2.0, 3.5]
    th = [0.3, 0.3 + math.pi]
    Fa = oracle.gabor_bank_iir(a, om, sg, th, "mirror")
    Fb = oracle.gabor_bank_iir(b, om, sg, th, "mirror")
    Fab = oracle.gabor_bank_iir((2 * a - 3 * b).astype(np.float32), om, sg, th, "mirror")
    np.testing.assert_allclose(Fab, 2 * Fa - 3 * Fb, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Fa[:, 1], np.conj(Fa[:, 0]), rtol=0, atol=1e-10)


@pytest.mark.parametrize("boundary", ["zero", "mirror"])
def test_approximates_the_direct_sum(boundary):
    img = workloads.smoothed_image(64, 72, 63)
    om, sg = [math.pi / 4, math.pi / 8], [2.0, 4.0]
    th = workloads.orientations(4)
    Fi = oracle.gabor_bank_iir(img, om, sg, th, boundary)
    Fd = oracle.gabor_bank(img, om, sg, th, 5.0, boundary)       # Gaussian to 5 sigma
    ser = 10 * np.log10((np.abs(Fd) ** 2).sum(axis=(2, 3)) / (np.abs(Fi - Fd) ** 2).sum(axis=(2, 3)))
    print("SER dB per channel", np.round(ser, 1))
    assert ser.min() > 27.0
