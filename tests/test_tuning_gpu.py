"""GPU checks of the schedule autotuner: tuning changes timing only, never
results; get/set round-trip; the JSON cache reapplies a stored schedule."""
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
    bank.close()
    cache = tuning.load_cache(path)
    assert len(cache) == 1 and list(cache.values())[0] == seg
    bank2 = gpu_lib.GaborBank(200, 300, [1.0, 0.3], [2.0, 6.0], 4, None, 3.0, "zero", "fp16_split")
    bank2.tuning = [32, 32]
    assert tuning.tuned(bank2, img, path=path) == seg      # a cache hit: no retuning
    assert bank2.tuning == seg
    bank2.close()
