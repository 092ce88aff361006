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
events that libgabor records on each launch's stream during a second timed
region of the same steps (the step time is taken without those events),
against the algorithmic work libgabor reports for that launch (the
four frequencies' launches run concurrently, so this time includes sharing
the chip); beside it, ``step`` is the whole step's algorithmic work over
``ms_per_step`` and ``isolated`` the same launch timed alone in a plan of its
one frequency.
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
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gabor-bank complex outputs/s, 1024² 8θ×4ω bank: FP32 plain vs BF16-MFMA form"
UNIT = "complex outputs/s"

# MI355X published peaks.  The FP32 vector figure is the unpacked rate (one
# FMA per lane per cycle: 256 CUs x 64 lanes x 2 flops x 2.4 GHz): libgabor is
# built without packed FP32 arithmetic, so the 157.3 TFLOP/s packed figure is
# out of its reach.
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp32_mfma": 157.3, "fp32_vector": 78.6, "bf16_mfma": 2500.0, "fp16_mfma": 2500.0}

FORMS = ["fp32", "bf16_split", "fp16_split", "bf16", "fp16", "fp32_twopass"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["paper_1704_05231_amd/csrc/gabor_ws.hip", "paper_1704_05231_amd/csrc/gabor_mfma.h",
                  "paper_1704_05231_amd/csrc/gabor_fused.hip", "paper_1704_05231_amd/csrc/gabor_fp32.hip"]
# HBM bytes of the box-window SDFT launch, from the same counters, keyed by its source
SDFT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sdft-box-512sq-16x16.json")
SDFT_SOURCES = ["paper_1704_05231_amd/csrc/gabor_sdft.hip"]
# the same for the localized SDFT launch (k_lsdft) and the recursive smoother
LSDFT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_lsdft-512sq-16x16.json")
LSDFT_SOURCES = ["paper_1704_05231_amd/csrc/gabor_ws.hip", "paper_1704_05231_amd/csrc/gabor_fused.hip",
                 "paper_1704_05231_amd/csrc/gabor_mfma.h", "paper_1704_05231_amd/csrc/gabor_lsdft.cpp"]
# the same for one adjoint call of the layer workload (k_adj_stream per frequency, k_adj_sum)
ADJ_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_layer-adjoint-32x512sq.json")
ADJ_SOURCES = ["paper_1704_05231_amd/csrc/gabor_fused.hip", "paper_1704_05231_amd/csrc/gabor_mfma.h",
               "paper_1704_05231_amd/csrc/gabor_plan.cpp"]
IIR_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_iir-bank-1024sq-8x4-mirror.json")
IIR_SOURCES = ["paper_1704_05231_amd/csrc/gabor_iir.hip"]


def source_hash(sources=None) -> str:
    h = hashlib.sha256()
    for rel in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(path, sources=None):
    """Per-kernel HBM bytes per launch from a counter summary, or None when
    the file is missing or the kernel sources changed since it was taken."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tf = json.load(fh)
    return tf.get("kernels", {}) if tf.get("source_hash") == source_hash(sources) else None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate host time for the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default=",".join(FORMS))
    ap.add_argument("--no-tune", action="store_true", help="keep the default segment heights")
    ap.add_argument("--workloads", default="lsdft,sdft,batch,layer,iir",
                    help="secondary workloads reported under 'workloads' (lsdft, sdft, batch, layer, iir; "
                         "empty: none)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run a plain device-to-device copy of MIB MiB instead (counter calibration)")
    ap.add_argument("--isolate", default="", metavar="FORMS",
                    help="instead of the bench line: run every frequency of the metric bank alone "
                         "(one single-frequency plan each, --steps launches, no concurrency) for each "
                         "listed form, and print their per-launch times (for counter runs)")
    ap.add_argument("--seg-rows", default="", metavar="S0,S1,..",
                    help="segment heights per frequency for every form timed (no autotuning) or, with "
                         "--isolate, for the isolated launches (default: autotuned / the plan's own)")
    ap.add_argument("--grouping", type=int, choices=(0, 1), default=None,
                    help="with --seg-rows: the plan's grouping option (1: the small operand sizes in one "
                         "launch; default: the plan's own)")
    return ap.parse_args()


def precision_of(form: str) -> str:
    return "fp32" if form == "fp32_twopass" else form


def time_form(binding, wl, img_dev, form, steps, warmup, tune=True, seg_rows=None, grouping=None):
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
    if seg_rows:
        bank.tuning = seg_rows
    if grouping is not None:
        bank.grouping = grouping
    tuning = bank.autotune(img_dev, out, reps=5) if tune and not seg_rows else bank.tuning
    grouping = bank.grouping
    for _ in range(warmup):
        bank(img_dev, out)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        bank(img_dev, out)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    # per-launch durations: a second timed region of the same steps with the
    # library's events around every launch (they cost about 10 us per step,
    # so the step time above is taken without them)
    bank.profile(True)
    for _ in range(steps):
        bank(img_dev, out)
    torch.cuda.synchronize()
    prof = bank.profile_read()
    bank.profile(False)
    info = bank.info
    res = out.cpu().numpy()
    bank.close()
    return ms, prof, info, res, tuning, grouping


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
    # traffic: HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE counters
    # (scaled by the copy calibration), null while the kernel sources differ
    # from the ones the counters were taken on
    r.update({"kernel": name, "traffic": t["hbm_bytes"] if t else None,
              "traffic_detail": t, "launch_ms": round(avg_s * 1e3, 5),
              "algorithmic_flops_per_launch": 2 * st["real_macs"],
              "algorithmic_bytes_per_launch": st["bytes"]})
    return r


def step_roofline(form, flops, nbytes, ms):
    """Whole-step figure: the step's algorithmic flops and bytes (image read
    once, every output written once) over the measured step time, against
    the roof that binds it."""
    kind, peak_c = ("alu", PEAK_TFLOPS["fp32_vector"]) if form == "fp32_twopass" else compute_peak(form, "")
    tflops, gbs = flops / (ms * 1e-3) / 1e12, nbytes / (ms * 1e-3) / 1e9
    fc, fm = tflops / peak_c, gbs / PEAK_HBM_GBS
    if fc >= fm:
        return {"bound": kind, "achieved": round(tflops, 3), "peak": peak_c, "unit": "TFLOP/s", "frac": round(fc, 4),
                "hbm_frac": round(fm, 4), "flops_per_step": flops, "bytes_per_step": nbytes, "ms_per_step": ms}
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(fm, 4),
            "compute_frac": round(fc, 4), "flops_per_step": flops, "bytes_per_step": nbytes, "ms_per_step": ms}


def launch_radii(name: str) -> list[int]:
    """Radii in a launch's profile name (ws_f32_r48 -> [48], ws_bf16_r12+24 -> [12, 24])."""
    return [int(v) for v in name.rsplit("_r", 1)[1].split("_")[0].split("+")]


def isolated_launch(binding, wl, img_dev, form, name, tuning, grouping, steps, warmup):
    """The launch `name` of the bank in a plan that holds only its frequency,
    launched alone: its event-timed average with no other launch sharing the
    chip, against the same per-launch algorithmic work."""
    import torch
    H, W = img_dev.shape
    radii = [int(math.ceil(wl.radius_sigmas * s - 1e-9)) for s in wl.sigmas]
    idx = [radii.index(R) for R in launch_radii(name)]
    if form == "fp32_twopass":
        os.environ["LIBGABOR_ALGO"] = "twopass"
    try:
        bank = binding.GaborBank(H, W, [wl.omegas[i] for i in idx], [wl.sigmas[i] for i in idx], wl.n_orient, None,
                                 wl.radius_sigmas, wl.boundary, precision_of(form))
    finally:
        os.environ.pop("LIBGABOR_ALGO", None)
    bank.tuning = [tuning[i] for i in idx]
    bank.grouping = grouping
    out = torch.empty((len(idx), wl.n_orient, H, W), dtype=torch.complex64, device="cuda")
    for _ in range(warmup):
        bank(img_dev, out)
    torch.cuda.synchronize()
    bank.profile(True)
    for _ in range(steps):
        bank(img_dev, out)
    torch.cuda.synchronize()
    st = bank.profile_read()[name]
    bank.profile(False)
    bank.close()
    avg_s = st["total_ms"] / st["launches"] * 1e-3
    tflops, gbs = 2.0 * st["real_macs"] / avg_s / 1e12, st["bytes"] / avg_s / 1e9
    kind, peak_c = compute_peak(form, name)
    fc, fm = tflops / peak_c, gbs / PEAK_HBM_GBS
    r = {"kernel": name, "launch_ms": round(avg_s * 1e3, 5), "segment_rows": [tuning[i] for i in idx]}
    if fc >= fm:
        r.update({"bound": kind, "achieved": round(tflops, 3), "peak": peak_c, "unit": "TFLOP/s", "frac": round(fc, 4)})
    else:
        r.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(fm, 4)})
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
    what = (f"every pixel ({n}, a whole step)" if n == H * W
            else f"{n} random pixels (corners included)")
    return {"value": n * n_ch / t, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{what} x {n_ch} channels of the same workload, FP64 direct Eq. (1), "
                      f"{t:.1f} s on {threads} threads",
            "cpu_model": host_cpu_model(), "host_cpus": os.cpu_count()}, xs, ys, ref


def host_cpu_model():
    """The host CPU's model name from /proc/cpuinfo (None where unreadable)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def event_time(fn, steps, warmup):
    """Average milliseconds of fn() over steps calls, HIP events on the
    current stream (every call here is one launch or a fixed launch group)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def hbm_roofline(nbytes, ms, note):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None, "basis": note}


def bench_lsdft(binding, workloads, steps, warmup):
    """512^2 uniform image, 16 x 16 window, sigma 4, all 256 bins, zero
    boundary: one lsdft_apply launch per step."""
    import oracle
    import torch
    wl = workloads.lsdft_512()
    img = torch.from_numpy(wl.image).cuda()
    H, W = wl.image.shape
    out = torch.empty((wl.my, wl.mx, H, W), dtype=torch.complex64, device="cuda")
    macs, nbytes = binding.lsdft_work(H, W, wl.my, wl.mx)
    xs, ys = workloads.sample_pixels(H, W, 300, 31)
    ref = oracle.lsdft_points(wl.image, wl.my, wl.mx, wl.sigma, xs, ys, wl.boundary)
    peak = np.abs(ref).max(0)
    # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters, per form
    traffic = load_traffic(LSDFT_TRAFFIC_FILE, LSDFT_SOURCES) or {}
    res = {"workload": wl.name, "outputs_per_call": wl.my * wl.mx * H * W, "forms": {}}
    for form in ["fp32", "fp16_split", "bf16_split", "bf16", "fp16"]:
        ms = event_time(lambda: binding.lsdft(img, wl.my, wl.mx, wl.sigma, wl.boundary, form, out=out),
                        steps * 4, warmup)
        got = out.cpu().numpy()[:, :, ys, xs].transpose(2, 0, 1)
        roof = hbm_roofline(nbytes, ms, "one launch per call")
        t = traffic.get(form)
        if t:
            roof.update({"traffic": t["hbm_bytes"], "traffic_detail": t})
        per_bin = np.abs(got - ref).max(0) / peak                 # [M_y, M_x], relative to each bin's peak
        worst = np.unravel_index(int(np.argmax(per_bin)), per_bin.shape)
        res["forms"][form] = {"ms": round(ms, 5), "value": wl.my * wl.mx * H * W / (ms * 1e-3),
                              "max_rel_err_per_bin": float(per_bin.max()),
                              "median_rel_err_per_bin": float(np.median(per_bin)),
                              "worst_bin_vu": [int(worst[0]), int(worst[1])],
                              "rel_err_per_bin": [[float("%.2g" % e) for e in row] for row in per_bin],
                              "roofline": roof}
    res["unit"] = UNIT
    res["algorithmic_bytes"] = nbytes
    res["algorithmic_real_macs"] = macs
    return res


def bench_sdft_box(binding, workloads, steps, warmup):
    """512^2 uniform image, 16 x 16 box window, all 256 bins, zero boundary:
    one sdft_box_apply launch per step (FP64 recursion, complex64 output)."""
    import oracle
    import torch
    wl = workloads.sdft_box_512()
    img = torch.from_numpy(wl.image).cuda()
    H, W = wl.image.shape
    out = torch.empty((wl.my, wl.mx, H, W), dtype=torch.complex64, device="cuda")
    nbytes = 4 * H * W + 8 * wl.my * wl.mx * H * W
    xs, ys = workloads.sample_pixels(H, W, 300, 33)
    ref = oracle.lsdft_points(wl.image, wl.my, wl.mx, wl.sigma, xs, ys, wl.boundary)
    ms = event_time(lambda: binding.sdft_box(img, wl.my, wl.mx, wl.boundary, out=out), steps * 4, warmup)
    got = out.cpu().numpy()[:, :, ys, xs].transpose(2, 0, 1)
    roof = hbm_roofline(nbytes, ms, "one launch per call")
    t = (load_traffic(SDFT_TRAFFIC_FILE, SDFT_SOURCES) or {}).get("k_sdft_box")
    if t:
        roof.update({"traffic": t["hbm_bytes"], "traffic_detail": t})
    return {"workload": wl.name, "outputs_per_call": wl.my * wl.mx * H * W, "unit": UNIT,
            "ms": round(ms, 5), "value": wl.my * wl.mx * H * W / (ms * 1e-3),
            "max_abs_err_over_max_f": float(np.abs(got - ref).max() / np.abs(wl.image).max()),
            "max_rel_err_per_bin": float((np.abs(got - ref).max(0) / np.abs(ref).max(0)).max()),
            "algorithmic_bytes": nbytes, "roofline": roof}


def bench_batch(binding, workloads, steps, warmup):
    """256 uniform images, sides uniform in [64, 1024], 8 orientations x 5
    frequencies pi/2 .. pi/32 (R up to 96), mirror: one gabor_batch_apply."""
    import oracle
    import torch
    from paper_1704_05231_amd import tuning
    wl = workloads.bank_batch()
    H = max(im.shape[0] for im in wl.images)
    W = max(im.shape[1] for im in wl.images)
    imgs = [torch.from_numpy(im).cuda() for im in wl.images]
    n_out = sum(im.shape[0] * im.shape[1] for im in wl.images) * len(wl.omegas) * wl.n_orient
    nbytes = sum(im.shape[0] * im.shape[1] for im in wl.images) * 4 + 8 * n_out
    res = {"workload": wl.name, "images": len(imgs), "outputs_per_call": n_out, "unit": UNIT, "forms": {}}
    for form in ["fp32", "bf16_split"]:
        bank = binding.GaborBank(H, W, wl.omegas, wl.sigmas, wl.n_orient, None, 3.0, wl.boundary, form)
        # schedule (segment heights, grouping option) tuned on whole batches;
        # results do not depend on it
        sched = tuning.tune_batch(bank, imgs)
        batch = binding.GaborBatch(bank, imgs)
        ms = event_time(batch, steps, warmup)
        n_launch, n_tiles = batch.info
        # the same batch captured once into a HIP graph and replayed
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            batch()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            batch()
        torch.cuda.synchronize()
        ms_graph = event_time(graph.replay, steps, warmup)
        worst = 0.0
        for i in (0, len(imgs) // 2, len(imgs) - 1):
            im = wl.images[i]
            xs, ys = workloads.sample_pixels(im.shape[0], im.shape[1], 64, 40 + i)
            ref = oracle.gabor_bank_points(im, wl.omegas, wl.sigmas, wl.thetas_or_default, xs, ys, 3.0,
                                           wl.boundary)
            got = batch.outputs[i].cpu().numpy()[:, :, ys, xs].transpose(2, 0, 1)
            worst = max(worst, float((np.abs(got - ref).max(0) / np.abs(ref).max(0)).max()))
        res["forms"][form] = {"ms": round(ms, 4), "value": n_out / (ms * 1e-3),
                              "ms_graph_replay": round(ms_graph, 4), "value_graph_replay": n_out / (ms_graph * 1e-3),
                              "launches": n_launch, "tiles": n_tiles, "schedule": sched,
                              "max_rel_err_sampled": worst,
                              "roofline": hbm_roofline(nbytes, ms_graph, "whole batch per graph replay "
                                                                         "(one launch per operand size)")}
        del graph
        batch.close()
        bank.close()
        del batch
        torch.cuda.empty_cache()
    return res


def bench_layer(binding, workloads, steps, warmup):
    """Differentiable layer: 32 uniform 512^2 images, the 8 x 4 bank, zero
    boundary; one forward and one backward (adjoint) of L = mean |F|^2."""
    import oracle
    import torch
    from paper_1704_05231_amd import tuning
    from paper_1704_05231_amd.autograd import GaborLayer
    wl = workloads.bank_layer()
    x0 = torch.from_numpy(np.stack(wl.images)).cuda()
    B, H, W = x0.shape
    layer = GaborLayer(H, W, wl.omegas, wl.sigmas, wl.n_orient)

    def step():
        # mean |F|^2 over all B x O x N x H x W outputs, as the squared
        # 2-norm of the interleaved (re, im) view over the output count: one
        # reading pass forward, one elementwise pass back
        x = x0.detach().requires_grad_(True)
        F = layer(x)
        (torch.linalg.vector_norm(torch.view_as_real(F)) ** 2 / F.numel()).backward()
        return x.grad

    # segment heights tuned on the whole step (forward and adjoint over the
    # batch); results do not depend on them
    sched = tuning.tune_step(layer.bank, step)
    ms = event_time(step, steps, warmup)
    g = step().cpu().numpy()
    layer.bank.profile(True)
    step()
    prof = layer.bank.profile_read()
    layer.bank.profile(False)
    xs, ys = workloads.sample_pixels(H, W, 8, 55)
    ref = oracle.gabor_grad_points(wl.images[0], wl.omegas, wl.sigmas, wl.thetas_or_default, xs, ys) / B
    err = float(np.abs(g[0][ys, xs] - ref).max() / np.abs(ref).max())
    # one batched adjoint call: the matrix-core adjoint (fused frequencies)
    # or the vector-ALU one, named adjoint_*_x<B>
    adj_name = next((k for k in prof if k.startswith("adjoint")), None)
    adj = prof.get(adj_name) if adj_name else None
    mfma = bool(adj_name) and adj_name.startswith("adjoint_mfma")
    adj_roof = None
    if adj:
        avg = adj["total_ms"] / adj["launches"]
        tf = 2 * adj["real_macs"] / (avg * 1e-3) / 1e12
        peak = PEAK_TFLOPS["fp32_mfma" if mfma else "fp32_vector"]
        adj_roof = {"bound": "mfma" if mfma else "alu", "achieved": round(tf, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(tf / peak, 4), "traffic": None,
                    "launch_ms": round(avg, 5),
                    "kernel": (f"{adj_name}: k_adj_stream, one launch per frequency over the batch, and the sum"
                               if mfma else f"{adj_name}: vector-ALU row + column passes")}
        # HBM bytes of the whole call from the counters under profiles/, while
        # the kernel sources match the hash they were taken on
        adj_tf = load_traffic(ADJ_TRAFFIC_FILE, ADJ_SOURCES) if mfma else None
        if adj_tf and "adjoint" in adj_tf:
            t = adj_tf["adjoint"]
            adj_roof["traffic"] = t["hbm_bytes"]
            adj_roof["traffic_detail"] = {"basis": "whole adjoint call", "fetch_bytes": t["fetch_bytes"],
                                          "write_bytes": t["write_bytes"], "algorithmic_bytes": t["algorithmic_bytes"],
                                          "ratio": t["ratio"]}
    layer.close()
    n_out = B * len(wl.omegas) * wl.n_orient * H * W
    fwd = {k: round(v["total_ms"] / v["launches"], 4) for k, v in prof.items() if not k.startswith("adjoint")}
    return {"workload": wl.name, "ms_forward_backward": round(ms, 4), "value": n_out / (ms * 1e-3),
            "unit": "complex outputs/s (forward + backward)", "grad_max_rel_err_vs_oracle": err,
            "forward_launch_ms": fwd, "adjoint_ms": round(adj["total_ms"] / adj["launches"], 4) if adj else None,
            "adjoint_roofline": adj_roof, "schedule": sched}


def bench_iir(binding, workloads, steps, warmup):
    """The metric workload's bank with the recursive smoother (modulate,
    third-order recursive Gaussian, demodulate; FP32): one gabor_bank_apply
    of an IIR plan per step, and its signal-to-error ratio against the direct
    Eq. (1) sum (Gaussian to 5 sigma) at sampled pixels."""
    import oracle
    import torch
    wl = workloads.bank_1024()
    img = wl.images[0]
    H, W = img.shape
    img_dev = torch.from_numpy(img).cuda()
    bank = binding.GaborBank(H, W, wl.omegas, wl.sigmas, wl.n_orient, None, 3.0, wl.boundary, "fp32",
                             smoother="iir")
    out = torch.empty((len(wl.omegas), wl.n_orient, H, W), dtype=torch.complex64, device="cuda")
    ms = event_time(lambda: bank(img_dev, out), steps, warmup)
    xs, ys = workloads.sample_pixels(H, W, 200, 57)
    ref = oracle.gabor_bank_points(img, wl.omegas, wl.sigmas, wl.thetas_or_default, xs, ys, 5.0, wl.boundary)
    got = out.cpu().numpy()[:, :, ys, xs].transpose(2, 0, 1)
    ser = 10 * np.log10((np.abs(ref) ** 2).sum(0) / (np.abs(got - ref) ** 2).sum(0))
    bank.close()
    n_out = len(wl.omegas) * wl.n_orient * H * W
    roof = hbm_roofline(4 * H * W + 8 * n_out, ms, "whole apply (every launch of the recursive smoother)")
    # HBM bytes of every launch of one apply, from the FETCH_SIZE / WRITE_SIZE counters
    t = (load_traffic(IIR_TRAFFIC_FILE, IIR_SOURCES) or {}).get("apply")
    if t:
        roof.update({"traffic": t["hbm_bytes"], "traffic_detail": t})
    return {"workload": wl.name + " (recursive smoother)", "ms": round(ms, 4), "value": n_out / (ms * 1e-3),
            "unit": UNIT, "ser_db_min": round(float(ser.min()), 2), "ser_db_max": round(float(ser.max()), 2),
            "roofline": roof}


def isolate(binding, wl, img_dev, forms, steps, warmup, seg_rows):
    """Each frequency of the bank in a plan of its own, launched alone
    `steps` times after `warmup`: per-launch event times with no other
    launch sharing the chip (the frequencies of an apply run concurrently)."""
    import torch
    H, W = img_dev.shape
    res = {}
    for form in forms:
        for i, (om, sg) in enumerate(zip(wl.omegas, wl.sigmas)):
            if form == "fp32_twopass":
                os.environ["LIBGABOR_ALGO"] = "twopass"
            try:
                bank = binding.GaborBank(H, W, [om], [sg], wl.n_orient, None, wl.radius_sigmas, wl.boundary,
                                         precision_of(form))
            finally:
                os.environ.pop("LIBGABOR_ALGO", None)
            if seg_rows:
                bank.tuning = [seg_rows[i]]
            out = torch.empty((1, wl.n_orient, H, W), dtype=torch.complex64, device="cuda")
            for _ in range(warmup):
                bank(img_dev, out)
            torch.cuda.synchronize()
            bank.profile(True)
            for _ in range(steps):
                bank(img_dev, out)
            torch.cuda.synchronize()
            prof = bank.profile_read()
            bank.profile(False)
            for name, st in prof.items():
                avg = st["total_ms"] / st["launches"]
                res[name] = {"form": form, "omega": om, "seg_rows": bank.tuning[0], "launches": st["launches"],
                             "avg_ms": round(avg, 5),
                             "tflops": round(2 * st["real_macs"] / (avg * 1e-3) / 1e12, 3),
                             "gbs": round(st["bytes"] / (avg * 1e-3) / 1e9, 1),
                             "real_macs": st["real_macs"], "bytes": st["bytes"]}
            bank.close()
            print(f"bench.py: isolated {form} omega={om:.4f} done", file=sys.stderr, flush=True)
    print(json.dumps({"isolated_launches": res, "workload": wl.name, "kernel_source_hash": source_hash()}),
          flush=True)


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

    traffic = load_traffic(TRAFFIC_FILE)

    wl = workloads.bank_1024()
    img = wl.images[0]
    H, W = img.shape
    n_out = len(wl.omegas) * wl.n_orient * H * W
    img_dev = torch.from_numpy(img).cuda()
    seg = [int(v) for v in args.seg_rows.split(",") if v]
    if seg and len(seg) != len(wl.omegas):
        sys.exit("bench.py: --seg-rows needs one height per frequency")
    if args.isolate:
        isolate(binding, wl, img_dev, [f for f in args.isolate.split(",") if f], args.steps, args.warmup, seg)
        return

    forms, results = {}, {}
    for form in [f for f in args.forms.split(",") if f]:
        ms, prof, info, res, tuning, grouping = time_form(binding, wl, img_dev, form, args.steps, args.warmup,
                                                          not args.no_tune, seg, args.grouping)
        results[form] = res
        forms[form] = {
            "value": n_out / (ms * 1e-3), "ms_per_step": round(ms, 5),
            "step_tflops": round(2.0 * info.real_macs / (ms * 1e-3) / 1e12, 3),
            "roofline": roofline_for(form, prof, traffic),
            "kernels": {k: {"launches": v["launches"], "avg_ms": round(v["total_ms"] / v["launches"], 5),
                            "real_macs": v["real_macs"], "bytes": v["bytes"]} for k, v in prof.items()},
            "real_macs_per_step": info.real_macs,
            "segment_rows": tuning,
            "grouping": grouping,
        }
        forms[form]["roofline"]["step"] = step_roofline(form, 2 * info.real_macs, 4 * H * W + 8 * n_out,
                                                        round(ms, 5))
        if form in ("fp32", "bf16_split"):
            forms[form]["roofline"]["isolated"] = isolated_launch(
                binding, wl, img_dev, form, forms[form]["roofline"]["kernel"], tuning, grouping, args.steps,
                args.warmup)
        print(f"bench.py: {form} done", file=sys.stderr, flush=True)

    cpu = None
    if forms and not args.no_cpu_baseline:
        cpu, xs, ys, ref = cpu_baseline(wl, img, args.cpu_seconds)
        peak = np.abs(ref).max(0)                                  # [O, N]
        for form, res in results.items():
            got = res[:, :, ys, xs].transpose(2, 0, 1)
            forms[form]["max_rel_err_vs_oracle"] = float((np.abs(got - ref).max(0) / peak).max())

    extra = {}
    for name in [w for w in args.workloads.split(",") if w]:
        extra[name] = {"lsdft": bench_lsdft, "sdft": bench_sdft_box, "batch": bench_batch, "layer": bench_layer, "iir": bench_iir}[name](
            binding, workloads, max(5, args.steps // 10), max(2, args.warmup // 5))
        print(f"bench.py: {name} done", file=sys.stderr, flush=True)
    if not forms:
        # secondary workloads only (--forms ""), e.g. for counter runs
        print(json.dumps({"workloads": extra, "kernel_source_hash": source_hash()}), flush=True)
        return
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
    if extra:
        line["workloads"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
