"""GPU checks of the schedule autotuner: tuning changes timing only, never
results; get/set round-trip; the JSON cache reapplies a stored schedule; the
grouping option (small operand sizes in one launch) keeps every bit."""
import math

import numpy as np
import pytest

from paper_1704_05231_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "bf16_split", "bf16", "fp16"])
def test_autotune_keeps_results_bitwise(gpu_lib, prec):
    import torch
    wl = workloads.bank_1024()
    bank = gpu_lib.GaborBank(1024, 1024, wl.omegas, wl.sigmas, 8, None, 3.0, "mirror", prec)
    img = torch.from_numpy(wl.images[0]).cuda()
    before = bank(img).clone()
    default = bank.tuning
    tuned = bank.autotune(img, reps=2)
    print(f"{prec}: default segments {default}, tuned {tuned}")
    assert all(v % 16 == 0 and v >= 16 for v in tuned)
    after = bank(img)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(before), torch.view_as_real(after))
    # a deliberately different schedule gives the same bits too
    bank.tuning = [32] * len(tuned)
    again = bank(img)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(before), torch.view_as_real(again))
    with pytest.raises(gpu_lib.GaborError):
        bank.tuning = [48] * len(tuned)
    with pytest.raises(gpu_lib.GaborError):
        bank.tuning = [128] * (len(tuned) + 1)
    bank.close()


def test_tuning_cache_round_trip(gpu_lib, tmp_path):
    import torch
    from paper_1704_05231_amd import tuning
    img = torch.from_numpy(workloads.uniform_image(200, 300, 800)).cuda()
    path = str(tmp_path / "tuning.json")
    bank = gpu_lib.GaborBank(200, 300, [1.0, 0.3], [2.0, 6.0], 4, None, 3.0, "zero", "fp16_split")
    seg = tuning.tuned(bank, img, reps=2, path=path)
    grouping = bank.grouping
    bank.close()
    cache = tuning.load_cache(path)
    assert len(cache) == 1 and list(cache.values())[0] == {"seg_rows": seg, "grouping": grouping}
    bank2 = gpu_lib.GaborBank(200, 300, [1.0, 0.3], [2.0, 6.0], 4, None, 3.0, "zero", "fp16_split")
    bank2.tuning = [32, 32]
    bank2.grouping = 1 - grouping
    assert tuning.tuned(bank2, img, path=path) == seg      # a cache hit: no retuning
    assert bank2.tuning == seg and bank2.grouping == grouping
    bank2.close()


# R = 6, 12, 24 (three small operand sizes in FP32, two in the 16-bit forms)
# and 48 (its own launch)
GROUP_OMEGAS = [math.pi / 2, math.pi / 4, math.pi / 8, math.pi / 16]
GROUP_SIGMAS = [2.0, 4.0, 8.0, 16.0]


@pytest.mark.parametrize("prec", ["fp32", "bf16_split", "fp16_split", "bf16", "fp16"])
def test_grouping_keeps_results_bitwise(gpu_lib, prec, monkeypatch):
    """The small quarters in one launch give the bits of one launch per
    quarter: through the cached apply graphs (dropped when the option
    changes), launch by launch, and in a batch of uneven images."""
    import torch
    H, W = 150, 210
    host = workloads.uniform_image(H, W, 810)
    img = torch.from_numpy(host).cuda()
    bank = gpu_lib.GaborBank(H, W, GROUP_OMEGAS, GROUP_SIGMAS, 8, None, 3.0, "mirror", prec)
    assert bank.grouping == 0
    bank.tuning = [32, 64, 96, 160]
    ref = bank(img).clone()
    for g in (1, 0, 1):
        bank.grouping = g
        assert bank.grouping == g
        for _ in range(2):                                     # first apply builds, second replays
            got = bank(img)
            torch.cuda.synchronize()
            assert torch.equal(torch.view_as_real(got), torch.view_as_real(ref)), f"grouping {g}"
    monkeypatch.setenv("LIBGABOR_NO_GRAPH", "1")
    eager = gpu_lib.GaborBank(H, W, GROUP_OMEGAS, GROUP_SIGMAS, 8, None, 3.0, "mirror", prec)
    eager.tuning = [32, 64, 96, 160]
    eager.grouping = 1
    got = eager(img)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(got), torch.view_as_real(ref))
    eager.close()
    monkeypatch.delenv("LIBGABOR_NO_GRAPH")
    with pytest.raises(gpu_lib.GaborError):
        bank.grouping = 2
    # a batch of uneven images under either option
    sizes = [(150, 210), (37, 53), (1, 90), (64, 1), (100, 130)]
    views = [torch.from_numpy(workloads.uniform_image(h, w, 820 + i)).cuda() for i, (h, w) in enumerate(sizes)]
    views[0] = img
    outs = {}
    for g in (0, 1):
        bank.grouping = g
        batch = gpu_lib.GaborBatch(bank, views)
        n_launch, _ = batch.info
        outs[g] = [o.clone() for o in batch()]
        torch.cuda.synchronize()
        # FP32: R = 6, 12, 24 share a launch; 16-bit forms: R = 12 and 24 already share a quarter
        assert n_launch == (4 if prec == "fp32" else 3) - (0 if g == 0 else (2 if prec == "fp32" else 1))
        batch.close()
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))
    assert torch.equal(torch.view_as_real(outs[0][0]), torch.view_as_real(ref))
    bank.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
def test_batch_tuner_keeps_results_bitwise(gpu_lib, prec):
    """tuning.tune_batch picks segment heights and the grouping option by
    timing whole batches; the batch's outputs keep every bit."""
    import torch
    from paper_1704_05231_amd import tuning
    sizes = [(150, 210), (37, 53), (1, 90), (64, 1), (100, 130), (150, 150)]
    views = [torch.from_numpy(workloads.uniform_image(h, w, 830 + i)).cuda() for i, (h, w) in enumerate(sizes)]
    bank = gpu_lib.GaborBank(150, 210, GROUP_OMEGAS, GROUP_SIGMAS, 8, None, 3.0, "mirror", prec)
    batch = gpu_lib.GaborBatch(bank, views)
    ref = [o.clone() for o in batch()]
    torch.cuda.synchronize()
    batch.close()
    sched = tuning.tune_batch(bank, views, reps=2)
    print(f"{prec}: batch schedule {sched}")
    assert sched["seg_rows"] == bank.tuning and sched["grouping"] == bank.grouping
    assert len(sched["candidates_ms"]) == 6
    batch = gpu_lib.GaborBatch(bank, views)
    got = batch()
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))
    batch.close()
    bank.close()


def test_step_tuner_keeps_layer_gradients_bitwise(gpu_lib):
    """tuning.tune_step picks segment heights by timing a whole layer step
    (forward and adjoint over a batch); the gradients keep every bit."""
    import torch
    from paper_1704_05231_amd import tuning
    from paper_1704_05231_amd.autograd import GaborLayer
    x0 = torch.from_numpy(np.stack([workloads.uniform_image(96, 112, 840 + i) for i in range(3)])).cuda()
    layer = GaborLayer(96, 112, GROUP_OMEGAS, GROUP_SIGMAS, 8)

    def step():
        x = x0.detach().requires_grad_(True)
        F = layer(x)
        (torch.linalg.vector_norm(torch.view_as_real(F)) ** 2 / F.numel()).backward()
        return x.grad

    ref = step().clone()
    sched = tuning.tune_step(layer.bank, step, reps=2)
    print(f"layer schedule {sched}")
    assert sched["seg_rows"] == layer.bank.tuning and len(sched["candidates_ms"]) == 3
    got = step()
    torch.cuda.synchronize()
    assert torch.equal(ref, got)
    layer.close()
