"""GPU checks of the strided-batch entry points: gabor_bank_apply_batched and
gabor_bank_apply_adjoint_batched give, image by image, the same bits as
gabor_bank_apply and gabor_bank_apply_adjoint (the same kernels and
schedules: a batch only adds the image index to the workgroup grid), on
padded image strides, both boundary rules, every form, plans whose
frequencies leave the wave-specialised kernel (one apply per image), mixed
matrix-core / vector-ALU adjoints and batches split into several groups."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PLANS = [
    # (H, W, omegas, sigmas, N)
    (64, 80, [math.pi / 4, math.pi / 8], [2.0, 3.0], 8),
    (37, 53, [1.3, 0.5], [1.5, 2.5], 5),
    (100, 120, [math.pi / 50, math.pi / 2], [25.0, 2.0], 4),   # R = 75 beside R = 6
]


def images(B, H, W, pad, seed):
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    buf = torch.full((B, H, W + pad), float("nan"), device="cuda")
    buf[:, :, :W] = torch.from_numpy(rng.uniform(0, 1, (B, H, W)).astype(np.float32)).cuda()
    return buf[:, :, :W]


@pytest.mark.parametrize("form", ["fp32", "bf16_split", "fp16"])
@pytest.mark.parametrize("boundary", ["zero", "mirror"])
@pytest.mark.parametrize("case", range(len(PLANS)))
def test_batched_forward_matches_single(gpu_lib, case, boundary, form):
    import torch
    H, W, om, sg, N = PLANS[case]
    bank = gpu_lib.GaborBank(H, W, om, sg, N, None, 3.0, boundary, form)
    x = images(3, H, W, 5, 700 + case)
    out = bank.apply_batched(x)
    torch.cuda.synchronize()
    for b in range(3):
        want = bank(x[b])
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(out[b]), torch.view_as_real(want)), f"image {b}"
    print(f"batched forward case {case} {boundary} {form}: {bank.tuning} bitwise equal")
    bank.close()


@pytest.mark.parametrize("boundary", ["zero", "mirror"])
@pytest.mark.parametrize("case", range(len(PLANS)))
def test_batched_adjoint_matches_single(gpu_lib, case, boundary, monkeypatch):
    import torch
    H, W, om, sg, N = PLANS[case]
    B = 5
    bank = gpu_lib.GaborBank(H, W, om, sg, N, None, 3.0, boundary, "fp32")
    rng = np.random.Generator(np.random.PCG64(720 + case))
    G = torch.from_numpy((rng.uniform(-1, 1, (B, len(om), N, H, W))
                          + 1j * rng.uniform(-1, 1, (B, len(om), N, H, W))).astype(np.complex64)).cuda()
    want = [bank.adjoint(G[b]).clone() for b in range(B)]
    torch.cuda.synchronize()
    got = bank.adjoint_batched(G)
    torch.cuda.synchronize()
    for b in range(B):
        assert torch.equal(got[b], want[b]), f"image {b}"
    # groups of two images (three groups), into padded gradient rows
    monkeypatch.setenv("LIBGABOR_ADJ_BATCH_BYTES", "1")
    buf = torch.full((B, H, W + 3), float("nan"), device="cuda")
    bank.adjoint_batched(G, buf[:, :, :W])
    torch.cuda.synchronize()
    for b in range(B):
        assert torch.equal(buf[b, :, :W], want[b]), f"image {b}, one per group"
    assert torch.isnan(buf[:, :, W:]).all()
    print(f"batched adjoint case {case} {boundary}: bitwise equal")
    bank.close()


def test_batched_empty_and_bad_strides(gpu_lib):
    import torch
    H, W, om, sg, N = PLANS[0]
    bank = gpu_lib.GaborBank(H, W, om, sg, N, None, 3.0, "zero", "fp32")
    x = images(2, H, W, 0, 730)
    out = torch.empty((2, 2, N, H, W), dtype=torch.complex64, device="cuda")
    gpu_lib.gabor_bank_apply_batched(bank._plan, x.data_ptr(), 0, x.stride(0), x.stride(1), out.data_ptr())
    with pytest.raises(gpu_lib.GaborError) as ei:        # images overlap
        gpu_lib.gabor_bank_apply_batched(bank._plan, x.data_ptr(), 2, W, x.stride(1), out.data_ptr())
    assert ei.value.status == 1
    with pytest.raises(gpu_lib.GaborError) as ei:
        gpu_lib.gabor_bank_apply_adjoint_batched(bank._plan, out.data_ptr(), 2, x.data_ptr(), W, W)
    assert ei.value.status == 1
    bank.close()


def test_layer_batch_graph_free_of_python_loops(gpu_lib):
    """The layer's batched forward and backward: one profiled launch per
    frequency forward (named _x<B>) and one adjoint launch group."""
    import torch
    from paper_1704_05231_amd.autograd import GaborLayer
    H, W, om, sg, N = PLANS[0]
    layer = GaborLayer(H, W, om, sg, N)
    x = images(4, H, W, 0, 740).contiguous().requires_grad_(True)
    layer.bank.profile(True)
    F = layer(x)
    (F.real ** 2 + F.imag ** 2).mean().backward()
    torch.cuda.synchronize()
    prof = layer.bank.profile_read()
    layer.bank.profile(False)
    names = sorted(prof)
    print("layer launches:", {k: v["launches"] for k, v in prof.items()})
    assert all(k.endswith("_x4") for k in names)
    assert sum(v["launches"] for k, v in prof.items() if k.startswith("ws_")) == 2
    assert sum(v["launches"] for k, v in prof.items() if k.startswith("adjoint")) == 1
    layer.close()
