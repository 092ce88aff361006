#!/usr/bin/env python3
"""Throughput of the 2-D complex Gabor filter bank on one MI355X.

Workload: one 1024 x 1024 smoothed-noise image (seeded), 8 orientations
k pi / 8, 4 frequencies pi/2, pi/4, pi/8, pi/16 with sigma = pi / omega
(2, 4, 8, 16 px; R = 3 sigma), mirror boundary, FP32 in, complex64 out:
33,554,432 complex outputs per step.  A step is one gabor_bank_apply over
the image already resident in HBM.

Prints one JSON line.  ``value`` is complex outputs per second of the FP32
form; the other arithmetic forms are reported beside it under ``forms``
(bf16_split is the matrix-core form that meets the 1e-3 bar).  ``roofline``
describes the launch that takes most of the FP32 step, timed live with HIP
events that libgabor records on each launch's stream during the timed
region, against the algorithmic work libgabor reports for that launch.
``cpu_baseline`` is the FP64 oracle (direct Eq. (1)) timed on the host on a
bounded random sample of the same workload's outputs, which also gives the
error of every form.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms a,b]
    python bench.py --calibrate-copy MIB    # plain device copy, for counters
"""
from __future__ import annotations

import argparse
import hashlib
import json
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
PEAK_TFLOPS = {"fp32_mfma": 157.3, "fp32_vector": 157.3, "bf16_mfma": 2500.0, "fp16_mfma": 2500.0}

FORMS = ["fp32", "bf16_split", "fp16_split", "bf16", "fp16", "fp32_twopass"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["paper_1704_05231_amd/csrc/gabor_fused.hip", "paper_1704_05231_amd/csrc/gabor_fp32.hip"]


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate host time for the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default=",".join(FORMS))
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run a plain device-to-device copy of MIB MiB instead (counter calibration)")
    return ap.parse_args()


def precision_of(form: str) -> str:
    return "fp32" if form == "fp32_twopass" else form


def time_form(binding, wl, img_dev, form, steps, warmup):
    import torch
    H, W = img_dev.shape
    if form == "fp32_twopass":
        os.environ["LIBGABOR_ALGO"] = "twopass"
    try:
        bank = binding.GaborBank(H, W, wl.omegas, wl.sigmas, wl.n_orient, None, wl.radius_sigmas,
                                 wl.boundary, precision_of(form))
    finally:
        os.environ.pop("LIBGABOR_ALGO", None)
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


def compute_peak(form: str, kernel: str) -> tuple[str, float]:
    if kernel.startswith(("row_fp32", "col_fp32")):
        return "alu", PEAK_TFLOPS["fp32_vector"]
    if form == "fp32":
        return "mfma", PEAK_TFLOPS["fp32_mfma"]
    return "mfma", PEAK_TFLOPS["bf16_mfma"]


def roofline_for(form, prof, traffic):
    """Launch with the largest total time: its algorithmic flops and bytes
    per launch over its event-timed average duration, against the roof that
    binds it (the larger of the two fractions)."""
    name, st = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    avg_s = st["total_ms"] / st["launches"] * 1e-3
    tflops = 2.0 * st["real_macs"] / avg_s / 1e12
    gbs = st["bytes"] / avg_s / 1e9
    unit_kind, peak_c = compute_peak(form, name)
    frac_c, frac_m = tflops / peak_c, gbs / PEAK_HBM_GBS
    t = traffic.get(name) if traffic else None
    if frac_c >= frac_m:
        r = {"bound": unit_kind, "achieved": round(tflops, 3), "peak": peak_c, "unit": "TFLOP/s",
             "frac": round(frac_c, 4), "other": {"unit": "GB/s", "achieved": round(gbs, 1),
                                                 "peak": PEAK_HBM_GBS, "frac": round(frac_m, 4)}}
    else:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "frac": round(frac_m, 4), "other": {"unit": "TFLOP/s", "achieved": round(tflops, 3),
                                                 "peak": peak_c, "frac": round(frac_c, 4)}}
    r.update({"kernel": name, "traffic": t, "launch_ms": round(avg_s * 1e3, 5),
              "algorithmic_flops_per_launch": 2 * st["real_macs"],
              "algorithmic_bytes_per_launch": st["bytes"]})
    return r


def cpu_baseline(wl, img, target_s):
    import oracle
    from paper_1704_05231_amd.workloads import sample_pixels
    thetas = wl.thetas_or_default
    n_ch = len(wl.omegas) * len(thetas)
    threads = oracle.max_threads()
    H, W = img.shape

    def run(n, seed):
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


def calibrate_copy(mib: int, steps: int):
    import torch
    n = mib * 1024 * 1024 // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    print(json.dumps({"calibrate_copy_bytes_read": 4 * n, "calibrate_copy_bytes_written": 4 * n,
                      "ms_per_copy": dt * 1e3, "gbs": 8 * n / dt / 1e9}), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, "
                  f"WORLD_SIZE={world}); the bank shards by image, frequency or row band with no "
                  f"collective, but no multi-GPU launch is built.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy, max(1, args.steps))
        return

    from paper_1704_05231_amd import binding, workloads
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    binding.load()

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tf = json.load(fh)
        if tf.get("source_hash") == source_hash():
            traffic = tf.get("kernels", {})

    wl = workloads.bank_1024()
    img = wl.images[0]
    H, W = img.shape
    n_out = len(wl.omegas) * wl.n_orient * H * W
    img_dev = torch.from_numpy(img).cuda()

    forms, results = {}, {}
    for form in [f for f in args.forms.split(",") if f]:
        ms, prof, info, res = time_form(binding, wl, img_dev, form, args.steps, args.warmup)
        results[form] = res
        forms[form] = {
            "value": n_out / (ms * 1e-3), "ms_per_step": round(ms, 5),
            "step_tflops": round(2.0 * info.real_macs / (ms * 1e-3) / 1e12, 3),
            "roofline": roofline_for(form, prof, traffic),
            "kernels": {k: {"launches": v["launches"], "avg_ms": round(v["total_ms"] / v["launches"], 5),
                            "real_macs": v["real_macs"], "bytes": v["bytes"]} for k, v in prof.items()},
            "real_macs_per_step": info.real_macs,
        }

    cpu = None
    if not args.no_cpu_baseline:
        cpu, xs, ys, ref = cpu_baseline(wl, img, args.cpu_seconds)
        peak = np.abs(ref).max(0)                                  # [O, N]
        for form, res in results.items():
            got = res[:, :, ys, xs].transpose(2, 0, 1)
            forms[form]["max_rel_err_vs_oracle"] = float((np.abs(got - ref).max(0) / peak).max())

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
        "kernel_source_hash": source_hash(),
    }
    if "bf16_split" in forms and "fp32" in forms:
        line["bf16_split_vs_fp32"] = round(forms["bf16_split"]["value"] / forms["fp32"]["value"], 3)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
