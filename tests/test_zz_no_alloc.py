"""GPU checks of gabor_bank_apply_adjoint_noalloc, the adjoint entry point
for callers that cannot allocate device memory: through the C ABI, its
gradient must equal the allocating gabor_bank_apply_adjoint's bit for bit
(same kernels, workspace from the library's fixed per-GPU array), on two
calls in a row (the second on a smaller plan, so the array holds the first
call's values), for both boundary rules and both adjoint paths; a plan that
needs more than the array returns GABOR_ERR_UNSUPPORTED and writes nothing."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

OMEGAS = [math.pi / 2, math.pi / 4, math.pi / 8, math.pi / 16]
SIGMAS = [math.pi / w for w in OMEGAS]


def _grads(gpu_lib, H, W, boundary, seed):
    import torch
    bank = gpu_lib.GaborBank(H, W, OMEGAS, SIGMAS, 8, None, 3.0, boundary, "fp32")
    rng = np.random.Generator(np.random.PCG64(seed))
    G = torch.from_numpy((rng.uniform(-1, 1, (4, 8, H, W)) + 1j * rng.uniform(-1, 1, (4, 8, H, W)))
                         .astype(np.complex64)).cuda()
    ref = torch.full((H, W), float("nan"), device="cuda")
    gpu_lib.gabor_bank_apply_adjoint(bank._plan, G.data_ptr(), ref.data_ptr(), W)
    out = torch.full((H, W), float("nan"), device="cuda")
    gpu_lib.gabor_bank_apply_adjoint_noalloc(bank._plan, G.data_ptr(), out.data_ptr(), W)
    torch.cuda.synchronize()
    bank.close()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("path,boundary", [("fused", "zero"), ("fused", "mirror"), ("twopass", "zero")])
def test_noalloc_adjoint_matches_allocating_adjoint(gpu_lib, path, boundary, monkeypatch):
    if path == "twopass":
        monkeypatch.setenv("LIBGABOR_ALGO", "twopass")
    # the layer workload's image size first, then a smaller, ragged one
    for (H, W, seed) in [(512, 512, 61), (200, 150, 62)]:
        print(f"noalloc adjoint {path} {boundary} {H}x{W}", flush=True)
        ref, out = _grads(gpu_lib, H, W, boundary, seed)
        assert np.isfinite(ref).all()
        np.testing.assert_array_equal(out, ref)


def test_noalloc_adjoint_rejects_plans_past_the_array(gpu_lib):
    import torch
    # 1024^2 with 20 jobs needs 80 MiB of partial planes (> 64 MiB)
    H = W = 1024
    bank = gpu_lib.GaborBank(H, W, OMEGAS, SIGMAS, 8, None, 3.0, "zero", "fp32")
    G = torch.zeros((4, 8, H, W), dtype=torch.complex64, device="cuda")
    out = torch.full((H, W), float("nan"), device="cuda")
    with pytest.raises(gpu_lib.GaborError) as e:
        gpu_lib.gabor_bank_apply_adjoint_noalloc(bank._plan, G.data_ptr(), out.data_ptr(), W)
    assert e.value.status == 4
    torch.cuda.synchronize()
    assert torch.isnan(out).all()
    bank.close()
