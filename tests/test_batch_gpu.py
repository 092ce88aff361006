"""GPU checks of the batched bank (gabor_batch_create / gabor_batch_apply):
uneven image sizes through one plan, bitwise agreement with the single-image
apply, the oracle, and HIP graph capture and replay."""
import math

import numpy as np
import pytest

import oracle
from bars import channel_bars
from paper_1704_05231_amd import workloads

pytestmark = pytest.mark.gpu

SIZES = [(37, 53), (64, 64), (1, 17), (100, 33), (9, 11), (70, 129), (23, 1), (128, 200)]
# R = 6, 24 and 60, all in the fused kernel; "fp32_twopass" forces the
# two-pass FP32 kernels (the path of R > 104) for every frequency
OMEGAS = [math.pi / 2, math.pi / 8, math.pi / 40]
SIGMAS = [2.0, 8.0, 20.0]
N = 6


def make_batch(gpu_lib, prec, boundary, sizes, seed0=600):
    import torch
    H = max(h for h, _ in sizes)
    W = max(w for _, w in sizes)
    bank = gpu_lib.GaborBank(H, W, OMEGAS, SIGMAS, N, None, 3.0, boundary, prec)
    host = [workloads.uniform_image(h, w, seed0 + i) for i, (h, w) in enumerate(sizes)]
    # every image in a wider buffer: row stride > width
    bufs = [torch.zeros((h, w + 5), dtype=torch.float32, device="cuda") for h, w in sizes]
    for b, im in zip(bufs, host):
        b[:, :im.shape[1]] = torch.from_numpy(im).cuda()
    views = [b[:, :w] for b, (h, w) in zip(bufs, sizes)]
    batch = gpu_lib.GaborBatch(bank, views)
    return bank, batch, host, views


@pytest.mark.parametrize("prec", ["fp32", "fp16_split", "bf16_split", "bf16", "fp32_twopass"])
@pytest.mark.parametrize("boundary", ["mirror", "zero"])
def test_batch_matches_single_image_and_oracle(gpu_lib, prec, boundary, monkeypatch):
    import torch
    twopass = prec == "fp32_twopass"
    if twopass:
        monkeypatch.setenv("LIBGABOR_ALGO", "twopass")
        prec = "fp32"
    bank, batch, host, views = make_batch(gpu_lib, prec, boundary, SIZES)
    outs = [o.cpu().numpy() for o in batch()]
    torch.cuda.synchronize()
    n_launch, n_tiles = batch.info
    # fused launches and their tiles (none when every frequency
    # takes the two-pass kernels)
    assert (n_launch, n_tiles) == (0, 0) if twopass else (n_launch >= 1 and n_tiles > 0)
    thetas = workloads.orientations(N)
    for i, (im, v) in enumerate(zip(host, views)):
        single = gpu_lib.GaborBank(im.shape[0], im.shape[1], OMEGAS, SIGMAS, N, None, 3.0, boundary, prec)
        ref_gpu = single(v).cpu().numpy()
        single.close()
        np.testing.assert_array_equal(outs[i], ref_gpu, err_msg=f"image {i} {im.shape}")
        ref = oracle.gabor_bank(im, OMEGAS, SIGMAS, thetas, 3.0, boundary)
        num = np.abs(outs[i] - ref).reshape(len(OMEGAS), N, -1).max(-1)
        den = np.abs(ref).reshape(len(OMEGAS), N, -1).max(-1)
        bar, nc = channel_bars(prec, float(np.abs(im).max()), den)
        ratio = num / np.maximum(bar, 1e-300)
        print(f"image {i} {im.shape}: max rel err {(num / den).max():.3e}, worst err/bar {ratio.max():.3f}, "
              f"{nc} cancelling channels")
        assert np.all(ratio <= 1), f"image {i}: {ratio.max():.3f}"
    batch.close()
    bank.close()


def test_batch_graph_capture_and_replay(gpu_lib):
    import torch
    bank, batch, host, views = make_batch(gpu_lib, "bf16_split", "mirror", SIZES[:5], seed0=700)
    eager = [o.clone() for o in batch()]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        batch()                                  # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        batch()
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(710))
    for rep in range(3):
        # new image contents between replays, plus eager work and syncs
        for v in views:
            v.copy_(torch.from_numpy(rng.uniform(0, 1, tuple(v.shape)).astype(np.float32)).cuda())
        for o in batch.outputs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        want = [o.clone() for o in batch()]
        torch.cuda.synchronize()
        for o in batch.outputs:
            o.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(batch.outputs, want):
            assert torch.equal(torch.view_as_real(a), torch.view_as_real(b)), f"replay {rep}"
    del eager
    batch.close()
    bank.close()


def test_single_apply_graph_capture_and_replay(gpu_lib):
    import torch
    wl = workloads.bank_1024()
    bank = gpu_lib.GaborBank(1024, 1024, wl.omegas, wl.sigmas, 8, None, 3.0, "mirror", "bf16_split")
    img = torch.from_numpy(wl.images[0]).cuda()
    out = torch.empty((4, 8, 1024, 1024), dtype=torch.complex64, device="cuda")
    want = bank(img).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bank(img, out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bank(img, out)
    for rep in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(out), torch.view_as_real(want)), f"replay {rep}"
    bank.close()


def test_batch_workload_sampled(gpu_lib):
    """The batched workload's first 16 images (sizes uniform in [64, 1024],
    8 orientations x 5 frequencies pi/2 .. pi/32, R up to 96, mirror),
    sampled against the oracle."""
    import torch
    wl = workloads.bank_batch(n=16)
    H = max(im.shape[0] for im in wl.images)
    W = max(im.shape[1] for im in wl.images)
    bank = gpu_lib.GaborBank(H, W, wl.omegas, wl.sigmas, wl.n_orient, None, 3.0, wl.boundary, "bf16_split")
    views = [torch.from_numpy(im).cuda() for im in wl.images]
    batch = gpu_lib.GaborBatch(bank, views)
    outs = batch()
    torch.cuda.synchronize()
    thetas = wl.thetas_or_default
    worst = 0.0
    for i in (0, 7, 15):
        im = wl.images[i]
        xs, ys = workloads.sample_pixels(im.shape[0], im.shape[1], 200, 720 + i)
        ref = oracle.gabor_bank_points(im, wl.omegas, wl.sigmas, thetas, xs, ys, 3.0, wl.boundary)
        got = outs[i].cpu().numpy()[:, :, ys, xs].transpose(2, 0, 1)
        err = (np.abs(got - ref).max(0) / np.abs(ref).max(0)).max()
        worst = max(worst, err)
    print(f"batch workload sampled max rel err {worst:.3e}")
    assert worst <= 1e-3
    batch.close()
    bank.close()
