#!/usr/bin/env python3
"""Throughput of the 2-D complex Gabor filter bank on one MI355X.

Workload: one 1024 x 1024 smoothed-noise image (seeded), 8 orientations
k pi / 8, 4 frequencies pi/2, pi/4, pi/8, pi/16 with sigma = pi / omega
(2, 4, 8, 16 px; R = 3 sigma), mirror boundary, FP32 in, complex64 out:
33,554,432 complex outputs per step.  A step is one gabor_bank_apply over
the image already resident in HBM.

Prints one JSON line.  ``value`` is complex outputs per second of the FP32
form; the matrix-core forms are reported beside it under ``forms``.
``roofline`` describes the kernel that takes most of the FP32 step, timed
live with HIP events recorded by libgabor on the launch stream during the
timed region.  ``cpu_baseline`` is the FP64 oracle (direct Eq. (1)) timed on
the host on a bounded random sample of the same workload's outputs.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gabor-bank complex outputs/s, 1024² 8θ×4ω bank: FP32 plain vs BF16-MFMA form"
UNIT = "complex outputs/s"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3     # with packed FP32; 78.6 without
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0

FORMS = ["fp32"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate host time for the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default=",".join(FORMS))
    return ap.parse_args()


def time_form(binding, wl, img_dev, precision, steps, warmup):
    import torch
    H, W = img_dev.shape
    bank = binding.GaborBank(H, W, wl.omegas, wl.sigmas, wl.n_orient, None, wl.radius_sigmas,
                             wl.boundary, precision)
    out = torch.empty((len(wl.omegas), wl.n_orient, H, W), dtype=torch.complex64, device="cuda")
    for _ in range(warmup):
        bank(img_dev, out)
    torch.cuda.synchronize()
    bank.profile(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        bank(img_dev, out)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    prof = bank.profile_read()
    bank.profile(False)
    info = bank.info
    res = out.cpu().numpy()
    bank.close()
    return ms, prof, info, res


def roofline_for(precision, prof, info, steps):
    """Dominant kernel of the step: its algorithmic flops per launch over its
    event-timed average launch duration, against the peak of the unit that
    bounds it."""
    name, (launches, total_ms) = max(prof.items(), key=lambda kv: kv[1][1])
    if name.startswith("row"):
        macs = info.row_real_macs
    elif name.startswith("col"):
        macs = info.col_real_macs
    else:
        macs = info.real_macs
    launches_per_step = launches / steps
    per_launch_ms = total_ms / launches
    flops_per_launch = 2.0 * macs / launches_per_step
    achieved = flops_per_launch / (per_launch_ms * 1e-3) / 1e12
    if precision == "fp32":
        bound, peak = "alu", PEAK_FP32_VECTOR_TFLOPS
    else:
        bound, peak = "mfma", PEAK_BF16_MFMA_TFLOPS
    return {"kernel": name, "bound": bound, "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
            "launch_ms": round(per_launch_ms, 5), "launches_per_step": launches_per_step,
            "algorithmic_flops_per_launch": flops_per_launch}


def cpu_baseline(wl, img, target_s):
    import oracle
    thetas = wl.thetas_or_default
    n_ch = len(wl.omegas) * len(thetas)
    threads = oracle.max_threads()
    H, W = img.shape

    def run(n, seed):
        from paper_1704_05231_amd.workloads import sample_pixels
        xs, ys = sample_pixels(H, W, n, seed)
        t0 = time.perf_counter()
        ref = oracle.gabor_bank_points(img, wl.omegas, wl.sigmas, thetas, xs, ys,
                                       wl.radius_sigmas, wl.boundary)
        return time.perf_counter() - t0, xs, ys, ref

    n0 = 4096
    t_small, *_ = run(n0, 7)
    n = int(min(H * W, max(n0, n0 * target_s / max(t_small, 1e-6))))
    t, xs, ys, ref = run(n, 8)
    return {"value": n * n_ch / t, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{n} random pixels (corners included) x {n_ch} channels of the same "
                      f"workload, FP64 direct Eq. (1), {t:.1f} s on {threads} threads"}, xs, ys, ref


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, "
                  f"WORLD_SIZE={world}); the path shards by image, frequency or row band "
                  f"with no collective, but no multi-GPU launch is built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_05231_amd import binding, workloads
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    binding.load()
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    wl = workloads.bank_1024()
    img = wl.images[0]
    H, W = img.shape
    n_out = len(wl.omegas) * wl.n_orient * H * W
    img_dev = torch.from_numpy(img).cuda()

    forms = {}
    results = {}
    for prec in [f for f in args.forms.split(",") if f]:
        ms, prof, info, res = time_form(binding, wl, img_dev, prec, args.steps, args.warmup)
        results[prec] = res
        forms[prec] = {"value": n_out / (ms * 1e-3), "ms_per_step": round(ms, 5),
                       "roofline": roofline_for(prec, prof, info, args.steps),
                       "kernels": {k: {"launches": v[0], "avg_ms": round(v[1] / v[0], 5)}
                                   for k, v in prof.items()},
                       "real_macs_per_step": info.real_macs}

    cpu = None
    if not args.no_cpu_baseline:
        cpu, xs, ys, ref = cpu_baseline(wl, img, args.cpu_seconds)
        peak = np.abs(ref).max(0)                                  # [O, N]
        for prec, res in results.items():
            got = res[:, :, ys, xs].transpose(2, 0, 1)
            forms[prec]["max_rel_err_vs_oracle"] = float((np.abs(got - ref).max(0) / peak).max())

    head = forms["fp32"] if "fp32" in forms else next(iter(forms.values()))
    line = {
        "metric": METRIC, "value": head["value"], "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "height": H, "width": W, "orientations": wl.n_orient,
                   "omegas": "pi/2,pi/4,pi/8,pi/16", "sigma": "pi/omega (2,4,8,16)",
                   "radius": "3 sigma (6,12,24,48)", "boundary": wl.boundary,
                   "outputs_per_step": n_out, "image": "5x5-box-smoothed uniform noise, seed 2"},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
