"""Seeded synthetic inputs and the workload parameter sets.

This module generates inputs only; it contains none of the filter arithmetic.
Both the GPU tests and the oracle-side tests draw their images here, so the
two implementations always see the same FP32 pixels.

The paper measures on 8-bit USC-SIPI photographs (1024 x 1024 for the bank
runtime table, 250 x 234 for the localized-SDFT table).  Those images are not
available; uniform [0, 1) pixels stand in for 8-bit intensities / 255, and
box-smoothed noise stands in for the spectral decay of natural images.  The
method has no data-dependent control flow, so throughput does not depend on
content; only the error magnitudes do.

Every generator uses numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ZERO = "zero"
MIRROR = "mirror"


def uniform_image(h: int, w: int, seed: int) -> np.ndarray:
    """i.i.d. uniform [0, 1) pixels, rounded to FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((h, w)).astype(np.float32)


def smoothed_image(h: int, w: int, seed: int) -> np.ndarray:
    """Uniform [0, 1) noise of (h+4) x (w+4), the valid 5 x 5 box mean, then
    min-max normalised to [0, 1]; FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((h + 4, w + 4))
    c = np.cumsum(np.cumsum(np.pad(u, ((1, 0), (1, 0))), axis=0), axis=1)
    box = (c[5:, 5:] - c[:-5, 5:] - c[5:, :-5] + c[:-5, :-5]) / 25.0
    lo, hi = box.min(), box.max()
    return ((box - lo) / (hi - lo)).astype(np.float32)


def orientations(n: int) -> np.ndarray:
    """theta_k = k pi / N, k = 0..N-1 (Sec. II-B)."""
    return np.array([math.pi * k / n for k in range(n)], dtype=np.float64)


@dataclass
class BankWorkload:
    name: str
    images: list                      # list of FP32 2-D arrays
    omegas: np.ndarray                # rad / px
    sigmas: np.ndarray                # px
    thetas: np.ndarray | None         # rad; None = k pi / N
    n_orient: int
    boundary: str
    radius_sigmas: float = 3.0
    meta: dict = field(default_factory=dict)

    @property
    def thetas_or_default(self) -> np.ndarray:
        return self.thetas if self.thetas is not None else orientations(self.n_orient)


@dataclass
class LsdftWorkload:
    name: str
    image: np.ndarray
    my: int
    mx: int
    sigma: float
    boundary: str


def bank_small(seed: int = 1) -> BankWorkload:
    """One 256 x 256 uniform image; orientations 0, 45, 90, 135 degrees;
    omega = pi/4, pi/8; sigma = 4 (25 x 25 taps); zero boundary."""
    return BankWorkload(
        name="bank-256sq-4x2-sigma4-zero",
        images=[uniform_image(256, 256, seed)],
        omegas=np.array([math.pi / 4, math.pi / 8]),
        sigmas=np.array([4.0, 4.0]),
        thetas=orientations(4),
        n_orient=4,
        boundary=ZERO,
    )


def bank_1024(seed: int = 2) -> BankWorkload:
    """One 1024 x 1024 smoothed-noise image; 8 orientations k pi / 8;
    omega = pi/2, pi/4, pi/8, pi/16 with sigma = 0.5 * 2 pi / omega
    (2, 4, 8, 16 px; R = 6, 12, 24, 48); mirror boundary."""
    om = np.array([math.pi / 2, math.pi / 4, math.pi / 8, math.pi / 16])
    return BankWorkload(
        name="bank-1024sq-8x4-mirror",
        images=[smoothed_image(1024, 1024, seed)],
        omegas=om,
        sigmas=0.5 * 2 * math.pi / om,
        thetas=None,
        n_orient=8,
        boundary=MIRROR,
    )


def lsdft_512(seed: int = 3) -> LsdftWorkload:
    """One 512 x 512 uniform image; 16 x 16 window, Gaussian sigma = 4;
    all 256 bins; zero boundary."""
    return LsdftWorkload("lsdft-512sq-16x16-sigma4", uniform_image(512, 512, seed),
                         16, 16, 4.0, ZERO)


# Window scale at which every Gaussian weight exp(-t^2 / (2 sigma^2)), |t| <= 64,
# rounds to exactly 1 in FP64: the localized SDFT with this sigma is the
# box-window SDFT.
BOX_SIGMA = 1e30


def sdft_box_512(seed: int = 3) -> LsdftWorkload:
    """The image of lsdft_512 (512 x 512 uniform); 16 x 16 box window; all
    256 bins; zero boundary.  sigma is BOX_SIGMA for the oracle."""
    return LsdftWorkload("sdft-box-512sq-16x16", uniform_image(512, 512, seed), 16, 16, BOX_SIGMA, ZERO)


def batch_sizes(n: int = 256, lo: int = 64, hi: int = 1024, seed: int = 4):
    """Side lengths drawn i.i.d. uniform on [lo, hi] inclusive (h, w independent)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [(int(h), int(w)) for h, w in rng.integers(lo, hi + 1, size=(n, 2))]


def bank_batch(n: int = 256, seed: int = 4) -> BankWorkload:
    """n uniform images of uneven sizes; 8 orientations; 5 frequencies
    pi/2 ... pi/32 (geometric), sigma = 0.5 * 2 pi / omega; mirror."""
    sizes = batch_sizes(n, seed=seed)
    imgs = [uniform_image(h, w, seed * 100003 + i) for i, (h, w) in enumerate(sizes)]
    om = np.array([math.pi / 2 ** (i + 1) for i in range(5)])
    return BankWorkload("bank-batch-uneven-8x5-mirror", imgs, om, 0.5 * 2 * math.pi / om,
                        None, 8, MIRROR, meta={"sizes": sizes})


def bank_layer(batch: int = 32, side: int = 512, seed: int = 5) -> BankWorkload:
    """A batch of uniform side x side images for the differentiable layer;
    the 8 x 4 bank of bank_1024 with zero boundary."""
    om = np.array([math.pi / 2, math.pi / 4, math.pi / 8, math.pi / 16])
    imgs = [uniform_image(side, side, seed * 1000 + i) for i in range(batch)]
    return BankWorkload("bank-layer-32x512sq-8x4-zero", imgs, om, 0.5 * 2 * math.pi / om,
                        None, 8, ZERO)


def sample_pixels(h: int, w: int, n: int, seed: int):
    """n distinct pixel coordinates (xs, ys) drawn uniformly, always including
    the four corners when n >= 4 (boundary handling is where errors hide)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.choice(h * w, size=min(n, h * w), replace=False)
    ys, xs = np.divmod(idx, w)
    if n >= 4 and h * w >= 4:
        ys[:4] = [0, 0, h - 1, h - 1]
        xs[:4] = [0, w - 1, 0, w - 1]
    return xs.astype(np.int32), ys.astype(np.int32)
