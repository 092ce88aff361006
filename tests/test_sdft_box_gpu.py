"""GPU parity of the box-window sliding DFT (the conventional SDFT of Sec. I;
Eq. (17) with a uniform window) through sdft_box_apply, against the FP64
oracle's localized SDFT at sigma = 1e30, where every window weight is
exactly 1/M (pinned against fft2 of the window patches on the CPU).

The kernel runs the circular-shift recursion in FP64 and re-anchors it by a
direct window sum every 8 columns, so its only single-precision step is the
final rounding to complex64.  Bar per output: 2^-23 |F_ref| (one rounding
of each component is at most 2^-24 |F_ref|; a factor 2 of slack) plus
1e-12 max|f| for the FP64 arithmetic."""
import numpy as np
import pytest

import oracle
from paper_1704_05231_amd import workloads

pytestmark = pytest.mark.gpu

BOX = workloads.BOX_SIGMA


def gpu_sdft(binding, img, my, mx, boundary="zero", stride_pad=0):
    import torch
    H, W = img.shape
    buf = torch.zeros((H, W + stride_pad), dtype=torch.float32, device="cuda")
    buf[:, :W] = torch.from_numpy(img).cuda()
    # poison the output: every plane must be overwritten
    out = torch.full((my, mx, H, W), float("nan"), dtype=torch.complex64, device="cuda")
    binding.sdft_box(buf[:, :W], my, mx, boundary, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(got, ref, img, what):
    assert np.all(np.isfinite(got)), "a bin plane was not written"
    err = np.abs(got - ref)
    bar = 2.0 ** -23 * np.abs(ref) + 1e-12 * float(np.abs(img).max())
    print(f"{what}: max err / max|f| {err.max() / np.abs(img).max():.3e}, worst err / bar {(err / bar).max():.3f}")
    assert np.all(err <= bar)


CASES = [
    # (H, W, My, Mx, boundary)
    (70, 150, 8, 8, "zero"),          # ragged run tail (150 = 18 runs of 8 + 6)
    (70, 150, 8, 8, "mirror"),
    (45, 77, 7, 7, "zero"),           # odd M: no real middle bin
    (45, 77, 12, 6, "mirror"),        # My != Mx
    (33, 40, 5, 10, "zero"),          # My < Mx
    (20, 19, 1, 1, "mirror"),         # one bin: the window average of one pixel
    (20, 19, 2, 2, "zero"),           # u, v in {0, M/2} only
    (1, 90, 4, 6, "mirror"),          # one row
    (90, 1, 6, 4, "zero"),            # one column: every update is a window shift past the edge
    (9, 1100, 4, 5, "mirror"),        # more than 512 columns: several passes of the 64 lanes
    (3, 5, 9, 11, "mirror"),          # window larger than the image (mirror folds repeatedly)
    (60, 70, 16, 16, "mirror"),       # the benchmark's window
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sdft_box_full_grid(gpu_lib, case):
    H, W, my, mx, bnd = CASES[case]
    img = workloads.uniform_image(H, W, 500 + case)
    got = gpu_sdft(gpu_lib, img, my, mx, bnd)
    ref = oracle.lsdft(img, my, mx, BOX, bnd)
    check(got, ref, img, f"sdft-box case {case} {H}x{W} {my}x{mx} {bnd}")


def test_sdft_box_conjugate_bins_bitwise(gpu_lib):
    """F_{Mx-u, My-v} = conj(F_{u,v}) for a real image: the kernel stores the
    conjugate of the very same values."""
    img = workloads.uniform_image(40, 70, 16)
    my, mx = 10, 6
    F = gpu_sdft(gpu_lib, img, my, mx, "mirror")
    for v in range(my):
        for u in range(mx):
            np.testing.assert_array_equal(F[(my - v) % my, (mx - u) % mx], np.conj(F[v, u]))


def test_sdft_box_row_stride(gpu_lib):
    img = workloads.uniform_image(50, 66, 17)
    a = gpu_sdft(gpu_lib, img, 8, 8, "mirror")
    b = gpu_sdft(gpu_lib, img, 8, 8, "mirror", stride_pad=9)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("shape", [(150, 170, 64, 64), (150, 170, 64, 3), (150, 170, 33, 64),
                                   (3, 8192, 4, 64)])
def test_sdft_box_limits_sampled(gpu_lib, shape):
    """Largest windows (M = 64) and the widest row (8192 columns, the FP64
    column DFTs filling on-chip memory), at sampled pixels."""
    H, W, my, mx = shape
    img = workloads.uniform_image(H, W, 18)
    xs, ys = workloads.sample_pixels(H, W, 40, 19)
    ref = oracle.lsdft_points(img, my, mx, BOX, xs, ys, "mirror")          # [P, My, Mx]
    got = gpu_sdft(gpu_lib, img, my, mx, "mirror")[:, :, ys, xs].transpose(2, 0, 1)
    check(got, ref, img, f"sdft-box {H}x{W} {my}x{mx} sampled")


def test_sdft_box_512_sampled(gpu_lib):
    """The 512^2, 16 x 16 box-window workload (all 256 bins) in its benchmark
    launch, at sampled pixels (corners included)."""
    wl = workloads.sdft_box_512()
    H, W = wl.image.shape
    xs, ys = workloads.sample_pixels(H, W, 1500, 20)
    ref = oracle.lsdft_points(wl.image, wl.my, wl.mx, wl.sigma, xs, ys, wl.boundary)
    got = gpu_sdft(gpu_lib, wl.image, wl.my, wl.mx, wl.boundary)[:, :, ys, xs].transpose(2, 0, 1)
    check(got, ref, wl.image, "sdft-box-512 sampled")


def test_sdft_box_graph_replays(gpu_lib):
    """Captured in a HIP graph and replayed three times, with eager work and
    synchronisation between replays: every replay equals the eager result."""
    import torch
    img = workloads.uniform_image(64, 96, 22)
    x = torch.from_numpy(img).cuda()
    eager = gpu_lib.sdft_box(x, 8, 8, "mirror")
    out = torch.empty_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gpu_lib.sdft_box(x, 8, 8, "mirror", out=out)          # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu_lib.sdft_box(x, 8, 8, "mirror", out=out)
    for _ in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)


def test_sdft_box_output_alignment(gpu_lib):
    """An output only 8-byte aligned (one complex64 element into a buffer)
    takes one-column stores; the values are the same bits as with the
    16-byte aligned output's two-column stores."""
    import torch
    img = workloads.uniform_image(30, 64, 23)
    x = torch.from_numpy(img).cuda()
    a = gpu_lib.sdft_box(x, 6, 8, "mirror")
    flat = torch.full((6 * 8 * 30 * 64 + 1,), float("nan"), dtype=torch.complex64, device="cuda")
    b = flat[1:].view(6, 8, 30, 64)
    assert b.data_ptr() % 16 == 8
    gpu_lib.sdft_box(x, 6, 8, "mirror", out=b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.isnan(flat[0]).item()


def draw(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    H = int(rng.integers(1, 25))
    W = int(rng.integers(1, 701))
    my, mx = int(rng.integers(1, 17)), int(rng.integers(1, 17))
    boundary = "mirror" if rng.integers(0, 2) else "zero"
    return H, W, my, mx, boundary


@pytest.mark.parametrize("seed", range(24))
def test_sdft_box_random_configuration(gpu_lib, seed):
    """Seeded random shapes (1..24 x 1..700: one or two 512-column chunks),
    windows (1..16 per axis) and boundary rules, every output against the
    oracle."""
    H, W, my, mx, bnd = draw(900 + seed)
    img = workloads.uniform_image(H, W, 1000 + seed)
    got = gpu_sdft(gpu_lib, img, my, mx, bnd)
    ref = oracle.lsdft(img, my, mx, BOX, bnd)
    check(got, ref, img, f"sdft-box seed {seed}: {H}x{W} {my}x{mx} {bnd}")
