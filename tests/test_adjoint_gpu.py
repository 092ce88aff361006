"""GPU checks of the hand-written adjoint (gabor_bank_apply_adjoint) and the
autograd layer built on it (FP32).

1. Dot-product identity: <bank(f), G> = <f, adjoint(G)> for random f and G,
   with <F, G> = sum Re(conj(G) F), both sides summed in FP64; both boundary
   rules (the mirror rule's adjoint is the transpose of the fold) on both
   adjoint paths, including images smaller than the band.
2. The oracle's FP64 gradient of L = mean |F|^2 at sampled pixels.
3. Central finite differences of the same loss (h = 1e-3) at sampled pixels,
   each difference formed as an FP64 sum over the outputs within R of the
   pixel, from two GPU forwards of the perturbed image (a difference of two
   whole-loss FP32 scalars would cancel below FP32 resolution).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1704_05231_amd import workloads

pytestmark = pytest.mark.gpu

BANKS = [
    # (H, W, omegas, sigmas, N, thetas)
    (64, 80, [math.pi / 4, math.pi / 8], [2.0, 3.0], 8, None),
    (37, 53, [1.3, 0.5], [1.5, 2.5], 5, None),                       # odd N: unpaired orientations
    (48, 40, [1.1], [2.2], 5, [0.0, 0.4, math.pi - 0.4, 1.0, math.pi / 2]),
    (20, 90, [0.0, 2.0], [3.0, 1.0], 3, None),                       # omega = 0
    (130, 70, [math.pi / 16], [16.0], 8, None),                      # R = 48 > half the width
    (9, 11, [0.9], [4.0], 5, None),                                  # R = 12 > both sides
    (1, 17, [1.0], [1.5], 3, None),                                  # one row
    (23, 1, [1.0, 0.3], [1.5, 2.0], 4, None),                        # one column
]


def make_bank(gpu_lib, H, W, om, sg, N, th, boundary="zero"):
    return gpu_lib.GaborBank(H, W, om, sg, N, th, 3.0, boundary, "fp32")


# "fused": the matrix-core adjoint of fused plans; "twopass": plans on the
# two-pass kernels take the vector-ALU adjoint (straight into dL/df under the
# zero boundary, one extended partial plane per frequency, folded, under the
# mirror rule)
@pytest.mark.parametrize("path,boundary", [("fused", "zero"), ("fused", "mirror"), ("twopass", "zero"),
                                           ("twopass", "mirror")])
@pytest.mark.parametrize("case", range(len(BANKS)))
def test_adjoint_dot_product_identity(gpu_lib, case, path, boundary, monkeypatch):
    import torch
    if path == "twopass":
        monkeypatch.setenv("LIBGABOR_ALGO", "twopass")
    H, W, om, sg, N, th = BANKS[case]
    bank = make_bank(gpu_lib, H, W, om, sg, N, th, boundary)
    rng = np.random.Generator(np.random.PCG64(500 + case))
    f = rng.uniform(-1, 1, (H, W)).astype(np.float32)
    G = (rng.uniform(-1, 1, (len(om), N, H, W)) + 1j * rng.uniform(-1, 1, (len(om), N, H, W))).astype(np.complex64)
    F = bank(torch.from_numpy(f).cuda()).cpu().numpy()
    g = bank.adjoint(torch.from_numpy(G).cuda()).cpu().numpy()
    bank.close()
    lhs = np.sum((np.conj(G.astype(np.complex128)) * F.astype(np.complex128)).real)
    rhs = np.sum(f.astype(np.float64) * g.astype(np.float64))
    scale = np.sum(np.abs(G) * np.abs(F))
    print(f"adjoint case {case} {path} {boundary}: <Ff,G> = {lhs:.9e}, <f,A G> = {rhs:.9e}, "
          f"rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_adjoint_row_stride_and_overwrite(gpu_lib):
    import torch
    H, W, om, sg, N, th = BANKS[0]
    bank = make_bank(gpu_lib, H, W, om, sg, N, th)
    rng = np.random.Generator(np.random.PCG64(510))
    G = torch.from_numpy((rng.uniform(-1, 1, (2, N, H, W)) + 1j * rng.uniform(-1, 1, (2, N, H, W)))
                         .astype(np.complex64)).cuda()
    a = bank.adjoint(G)
    buf = torch.full((H, W + 7), float("nan"), device="cuda")
    b = bank.adjoint(G, buf[:, :W])
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.isnan(buf[:, W:]).all()          # padding columns untouched
    bank.close()


def loss_grad_gpu(gpu_lib, img, om, sg, N, th, boundary="zero"):
    """Autograd gradient of L = mean |F|^2 through the layer."""
    import torch
    from paper_1704_05231_amd.autograd import GaborLayer
    H, W = img.shape
    layer = GaborLayer(H, W, om, sg, N, th, boundary=boundary)
    x = torch.from_numpy(img).cuda().requires_grad_(True)
    F = layer(x)
    loss = (F.real ** 2 + F.imag ** 2).mean()
    loss.backward()
    g = x.grad.cpu().numpy()
    layer.close()
    return g


@pytest.mark.parametrize("case", [0, 1, 3, 4])
def test_autograd_gradient_matches_oracle(gpu_lib, case):
    H, W, om, sg, N, th = BANKS[case]
    img = workloads.uniform_image(H, W, 520 + case)
    thetas = workloads.orientations(N) if th is None else np.asarray(th)
    g = loss_grad_gpu(gpu_lib, img, om, sg, N, th)
    xs, ys = workloads.sample_pixels(H, W, 64, 530 + case)
    ref = oracle.gabor_grad_points(img, om, sg, thetas, xs, ys)
    err = np.abs(g[ys, xs] - ref).max() / np.abs(ref).max()
    print(f"grad case {case}: max err / peak {err:.2e}")
    assert err <= 1e-5


def test_autograd_gradient_matches_finite_differences(gpu_lib):
    import torch
    H, W = 96, 112
    om, sg, N = [math.pi / 2, math.pi / 4], [2.0, 4.0], 8
    img = workloads.uniform_image(H, W, 540)
    g = loss_grad_gpu(gpu_lib, img, om, sg, N, None)
    bank = gpu_lib.GaborBank(H, W, om, sg, N, None, 3.0, "zero", "fp32")
    n = len(om) * N * H * W
    R = int(math.floor(3 * max(sg) + 0.5))
    h = 1e-3
    xs, ys = workloads.sample_pixels(H, W, 24, 541)
    fd = np.empty(len(xs))
    for i, (x, y) in enumerate(zip(xs, ys)):
        vals = []
        for s in (+1, -1):
            pert = img.copy()
            pert[y, x] += s * h
            F = bank(torch.from_numpy(pert).cuda()).cpu().numpy()
            win = F[:, :, max(0, y - R):y + R + 1, max(0, x - R):x + R + 1].astype(np.complex128)
            vals.append(np.sum(np.abs(win) ** 2) / n)
        fd[i] = (vals[0] - vals[1]) / (2 * h)
    bank.close()
    err = np.abs(fd - g[ys, xs]).max() / np.abs(g[ys, xs]).max()
    print(f"finite differences: max err / peak {err:.2e}")
    assert err <= 5e-3


def test_autograd_mirror_gradient_matches_finite_differences(gpu_lib):
    # Under the mirror rule a pixel near an edge also feeds the outputs near
    # its reflections, so each difference sums |F|^2 over every output (in
    # FP64; the unchanged outputs are bitwise equal in both runs and cancel).
    import torch
    H, W = 48, 56
    om, sg, N = [math.pi / 2, math.pi / 4], [2.0, 4.0], 8
    img = workloads.uniform_image(H, W, 545)
    g = loss_grad_gpu(gpu_lib, img, om, sg, N, None, "mirror")
    bank = gpu_lib.GaborBank(H, W, om, sg, N, None, 3.0, "mirror", "fp32")
    n = len(om) * N * H * W
    h = 1e-3
    xs, ys = workloads.sample_pixels(H, W, 16, 546)
    fd = np.empty(len(xs))
    for i, (x, y) in enumerate(zip(xs, ys)):
        vals = []
        for sgn in (+1, -1):
            pert = img.copy()
            pert[y, x] += sgn * h
            F = bank(torch.from_numpy(pert).cuda()).cpu().numpy().astype(np.complex128)
            vals.append(np.sum(np.abs(F) ** 2) / n)
        fd[i] = (vals[0] - vals[1]) / (2 * h)
    bank.close()
    err = np.abs(fd - g[ys, xs]).max() / np.abs(g[ys, xs]).max()
    print(f"mirror finite differences: max err / peak {err:.2e}")
    assert err <= 5e-3


def test_feature_layer_workload_sampled(gpu_lib):
    """The differentiable-layer workload: a batch of 32 uniform 512^2 images,
    8 orientations x 4 frequencies (sigma = pi / omega), zero boundary,
    L = mean |F|^2 over the batch; gradients of the first and last image
    checked against the oracle at sampled pixels."""
    import torch
    from paper_1704_05231_amd.autograd import GaborLayer
    wl = workloads.bank_layer()
    imgs = np.stack(wl.images)
    B, H, W = imgs.shape
    layer = GaborLayer(H, W, wl.omegas, wl.sigmas, wl.n_orient)
    x = torch.from_numpy(imgs).cuda().requires_grad_(True)
    F = layer(x)
    loss = (F.real ** 2 + F.imag ** 2).mean()
    loss.backward()
    g = x.grad.cpu().numpy()
    layer.close()
    thetas = wl.thetas_or_default
    for b in (0, B - 1):
        xs, ys = workloads.sample_pixels(H, W, 8, 550 + b)
        # the oracle's loss is the mean over one image's outputs: scale by 1/B
        ref = oracle.gabor_grad_points(imgs[b], wl.omegas, wl.sigmas, thetas, xs, ys) / B
        err = np.abs(g[b][ys, xs] - ref).max() / np.abs(ref).max()
        print(f"layer image {b}: max err / peak {err:.2e}")
        assert err <= 1e-5


def test_feature_layer_finite_differences_64_pixels(gpu_lib):
    """The layer workload's gradient check: one 512^2 image of the batch
    (seed 5, zero boundary, 8 x 4 bank, sigma = pi / omega), L = mean |F|^2
    over its outputs, central differences with h = 1e-3 at 64 seeded pixels.
    Each difference sums |F|^2 in FP64 over the outputs within R of the pixel
    (the others are bitwise equal in the two forwards and cancel); L is
    quadratic, so the central difference has no truncation error and the
    bar is set by the FP32 outputs' rounding."""
    import torch
    wl = workloads.bank_layer()
    img = wl.images[0]
    H, W = img.shape
    g = loss_grad_gpu(gpu_lib, img, wl.omegas, wl.sigmas, wl.n_orient, None)
    bank = gpu_lib.GaborBank(H, W, wl.omegas, wl.sigmas, wl.n_orient, None, 3.0, "zero", "fp32")
    n = len(wl.omegas) * wl.n_orient * H * W
    R = int(math.floor(3 * max(wl.sigmas) + 0.5))
    h = 1e-3
    xs, ys = workloads.sample_pixels(H, W, 64, 105)
    base = torch.from_numpy(img).cuda()
    fd = np.empty(len(xs))
    for i, (x, y) in enumerate(zip(xs, ys)):
        vals, steps = [], []
        for sgn in (+1, -1):
            # the step the FP32 image actually takes (f + h rounds)
            v = np.float32(img[y, x] + np.float32(sgn * h))
            steps.append(abs(float(v) - float(img[y, x])))
            pert = base.clone()
            pert[y, x] = float(v)
            F = bank(pert)[:, :, max(0, y - R):y + R + 1, max(0, x - R):x + R + 1]
            vals.append(float(torch.sum(torch.abs(F.to(torch.complex128)) ** 2)) / n)
        fd[i] = (vals[0] - vals[1]) / (steps[0] + steps[1])
    bank.close()
    err = np.abs(fd - g[ys, xs]).max() / np.abs(g[ys, xs]).max()
    print(f"layer 512^2 finite differences at 64 pixels: max err / peak {err:.2e}")
    assert err <= 1e-4


def draw(seed):
    """Shape, frequencies, radii, orientations and rule; radii up to 56 take
    the matrix-core adjoint, larger ones the vector-ALU one (mixed plans take
    both, one per frequency)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W = int(rng.integers(1, 80)), int(rng.integers(1, 90))
    boundary = "mirror" if rng.integers(0, 2) else "zero"
    choices = [0, 1, 3, 6, 10, 20, 27, 30, 40, 45, 56, 70, 88, 104, 110]
    n_freq = int(rng.integers(1, 3))
    radii = [int(rng.choice(choices)) for _ in range(n_freq)]
    sigmas = [r / 3.0 if r > 0 else 0.1 for r in radii]
    omegas = [float(rng.uniform(0.0, math.pi)) for _ in range(n_freq)]
    return H, W, omegas, sigmas, int(rng.integers(1, 9)), boundary


@pytest.mark.parametrize("seed", range(24))
def test_adjoint_random_dot_product_identity(gpu_lib, seed):
    """<bank(f), G> = <f, adjoint(G)> over seeded random configurations."""
    import torch
    H, W, om, sg, N, bnd = draw(540 + seed)
    bank = make_bank(gpu_lib, H, W, om, sg, N, None, bnd)
    rng = np.random.Generator(np.random.PCG64(560 + seed))
    f = rng.uniform(-1, 1, (H, W)).astype(np.float32)
    G = (rng.uniform(-1, 1, (len(om), N, H, W)) + 1j * rng.uniform(-1, 1, (len(om), N, H, W))).astype(np.complex64)
    F = bank(torch.from_numpy(f).cuda()).cpu().numpy()
    g = bank.adjoint(torch.from_numpy(G).cuda()).cpu().numpy()
    bank.close()
    lhs = np.sum((np.conj(G.astype(np.complex128)) * F.astype(np.complex128)).real)
    rhs = np.sum(f.astype(np.float64) * g.astype(np.float64))
    scale = np.sum(np.abs(G) * np.abs(F))
    radii = [int(math.floor(3 * s + 0.5)) for s in sg]
    print(f"adjoint seed {seed}: {H}x{W} N={N} R={radii} {bnd}: rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-6 * scale


def mirror_fd(gpu_lib, img, om, sg, N, n_px, seed, h):
    """Central differences (step h, the FP32 image's actual steps) of
    L = mean |F|^2 under the mirror rule, summing |F|^2 over every output
    in FP64 (the outputs the pixel does not reach are bitwise equal in the
    two forwards and cancel)."""
    import torch
    H, W = img.shape
    bank = gpu_lib.GaborBank(H, W, om, sg, N, None, 3.0, "mirror", "fp32")
    n = len(om) * N * H * W
    xs, ys = workloads.sample_pixels(H, W, n_px, seed)
    base = torch.from_numpy(img).cuda()
    fd = np.empty(len(xs))
    for i, (x, y) in enumerate(zip(xs, ys)):
        vals, steps = [], []
        for sgn in (+1, -1):
            v = np.float32(img[y, x] + np.float32(sgn * h))
            steps.append(abs(float(v) - float(img[y, x])))
            pert = base.clone()
            pert[y, x] = float(v)
            F = bank(pert)
            vals.append(float(torch.sum(torch.abs(F.to(torch.complex128)) ** 2)) / n)
        fd[i] = (vals[0] - vals[1]) / (steps[0] + steps[1])
    bank.close()
    return fd, xs, ys


@pytest.mark.parametrize("R", [75, 96])
def test_adjoint_mirror_large_radius(gpu_lib, R):
    """Mirror rule beyond the matrix-core adjoint's reach (R = 75, 96: the
    vector-ALU adjoint on the image extended by R, folded back; R = 96 is
    larger than the image's half-width, so positions fold more than once),
    beside a matrix-core frequency: dot-product identity, then the layer's
    gradient against central finite differences at 16 pixels.  L is
    quadratic in f, so a central difference has no truncation error at any
    step: h = 0.25 keeps the FP32 rounding of the roughly 2 x 10^5 outputs a
    pixel reaches at R = 96 (their |F|^2 summed twice) well below the
    difference itself, where h = 1e-3 leaves it near 1e-3 of the peak."""
    import torch
    H, W = 100, 120
    sg = [R / 3.0, 2.0]
    om = [math.pi / (2 * sg[0]), math.pi / 2]
    N = 4
    bank = make_bank(gpu_lib, H, W, om, sg, N, None, "mirror")
    rng = np.random.Generator(np.random.PCG64(600 + R))
    f = rng.uniform(-1, 1, (H, W)).astype(np.float32)
    G = (rng.uniform(-1, 1, (2, N, H, W)) + 1j * rng.uniform(-1, 1, (2, N, H, W))).astype(np.complex64)
    F = bank(torch.from_numpy(f).cuda()).cpu().numpy()
    g = bank.adjoint(torch.from_numpy(G).cuda()).cpu().numpy()
    bank.close()
    lhs = np.sum((np.conj(G.astype(np.complex128)) * F.astype(np.complex128)).real)
    rhs = np.sum(f.astype(np.float64) * g.astype(np.float64))
    scale = np.sum(np.abs(G) * np.abs(F))
    print(f"mirror R={R}: dot-product rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-6 * scale
    img = workloads.uniform_image(H, W, 610 + R)
    grad = loss_grad_gpu(gpu_lib, img, om, sg, N, None, "mirror")
    fd, xs, ys = mirror_fd(gpu_lib, img, om, sg, N, 16, 620 + R, 0.25)
    err = np.abs(fd - grad[ys, xs]).max() / np.abs(grad[ys, xs]).max()
    print(f"mirror R={R} finite differences: max err / peak {err:.2e}")
    assert err <= 1e-4
