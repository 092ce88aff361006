"""GPU checks of gabor_bank_apply's cached graphs: an apply is captured once
per (image, stride, output, segment heights) and replayed afterwards.  The
replays must give the bits of the launch-by-launch submission
(LIBGABOR_NO_GRAPH=1), follow new image contents, survive more buffer
triples than the cache holds (evictions), and follow a schedule change."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_graph_replays_match_launch_by_launch(gpu_lib, monkeypatch):
    import torch
    H, W = 96, 130
    om, sg = [math.pi / 4, math.pi / 16], [2.0, 16.0]
    rng = np.random.Generator(np.random.PCG64(760))
    imgs = [torch.from_numpy(rng.uniform(0, 1, (H, W)).astype(np.float32)).cuda() for _ in range(6)]
    for form in ["fp32", "bf16_split"]:
        monkeypatch.setenv("LIBGABOR_NO_GRAPH", "1")
        ref_bank = gpu_lib.GaborBank(H, W, om, sg, 8, None, 3.0, "mirror", form)
        monkeypatch.delenv("LIBGABOR_NO_GRAPH")
        bank = gpu_lib.GaborBank(H, W, om, sg, 8, None, 3.0, "mirror", form)
        outs = [torch.full((2, 8, H, W), float("nan"), dtype=torch.complex64, device="cuda") for _ in imgs]
        want = [ref_bank(im).clone() for im in imgs]
        # six buffer pairs through a cache of four, twice: captures, hits and evictions
        for rep in range(2):
            for im, o in zip(imgs, outs):
                o.fill_(float("nan"))
                bank(im, o)
            torch.cuda.synchronize()
            for k, (o, w) in enumerate(zip(outs, want)):
                assert torch.equal(torch.view_as_real(o), torch.view_as_real(w)), f"{form} rep {rep} buffer {k}"
        # new contents in a cached buffer
        imgs[0].mul_(0.5).add_(0.25)
        bank(imgs[0], outs[0])
        w0 = ref_bank(imgs[0])
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(outs[0]), torch.view_as_real(w0)), f"{form} new contents"
        # a schedule change is a new graph
        seg = [32, 64]
        bank.tuning = seg
        ref_bank.tuning = seg
        bank(imgs[1], outs[1])
        w1 = ref_bank(imgs[1])
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(outs[1]), torch.view_as_real(w1)), f"{form} after retuning"
        bank.close()
        ref_bank.close()
