"""JSON cache of autotuned schedules.

``tuned(bank, img)`` looks the bank's configuration up in the cache (keyed by
GPU name, library build and every plan parameter); on a miss it runs
``gabor_bank_autotune`` on ``img`` and stores the result.  The cache lives in
``$LIBGABOR_TUNING_CACHE`` or ``~/.cache/libgabor/tuning.json``.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import binding


def cache_path() -> str:
    return os.environ.get("LIBGABOR_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "libgabor", "tuning.json"))


def _library_id() -> str:
    h = hashlib.sha256()
    with open(os.environ.get("LIBGABOR_LIBRARY", binding.LIB_PATH), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def key(bank) -> str:
    import torch
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(dev, "gcnArchName", "")
    return json.dumps({"gpu": dev.name, "arch": arch, "lib": _library_id(), **bank.params}, sort_keys=True)


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def store_cache(cache: dict, path: str | None = None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(bank, img, out=None, reps: int = 5, path: str | None = None) -> list[int]:
    """Apply the cached schedule of this bank (segment heights and grouping
    option), or tune and cache it; returns the segment heights."""
    cache = load_cache(path)
    k = key(bank)
    entry = cache.get(k)
    if isinstance(entry, dict) and "seg_rows" in entry:
        bank.tuning = entry["seg_rows"]
        bank.grouping = int(entry.get("grouping", 0))
        return entry["seg_rows"]
    seg = bank.autotune(img, out, reps)
    cache[k] = {"seg_rows": seg, "grouping": bank.grouping}
    store_cache(cache, path)
    return seg


def tune_batch(bank, images, reps: int = 3, mults=(1, 2, 4)) -> dict:
    """Schedule of a batch of uneven images (segment heights and grouping
    option) by timing whole batches: the bank's current heights scaled by
    each of `mults` (capped at the plan height), under both grouping
    settings; the fastest is applied to the bank.  With many images there is
    parallelism enough for longer segments (less lead-in) than a single
    image's tuning picks.  Results do not depend on the choice.  Returns the
    chosen schedule and every candidate's time (ms, median of `reps` timed
    batches after one warm-up)."""
    import torch
    base = bank.tuning
    hmax = (bank.height + 15) // 16 * 16
    times = {}
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def scaled(m):
        # frequencies on the two-pass kernels report 0 and take any height
        return [min(s * m, hmax) if s else hmax for s in base]

    for g in (0, 1):
        for m in mults:
            bank.tuning = scaled(m)
            bank.grouping = g
            batch = binding.GaborBatch(bank, images)
            batch()
            ts = []
            for _ in range(reps):
                start.record()
                batch()
                stop.record()
                stop.synchronize()
                ts.append(start.elapsed_time(stop))
            batch.close()
            times[(g, m)] = sorted(ts)[len(ts) // 2]
    g, m = min(times, key=times.get)
    bank.tuning = scaled(m)
    bank.grouping = g
    return {"seg_rows": bank.tuning, "grouping": g,
            "candidates_ms": {f"grouping {gg}, x{mm}": round(t, 4) for (gg, mm), t in times.items()}}


def tune_step(bank, step, reps: int = 5, mults=(1, 2, 4)) -> dict:
    """Segment heights for a caller's whole step (for example a layer's
    forward and adjoint over a batch): `step()` is timed with the bank's
    current heights scaled by each of `mults` (capped at the plan height),
    the median of `reps` timed calls after one warm-up, and the fastest
    heights are applied.  Results do not depend on the choice.  Returns the
    chosen heights and every candidate's time (ms)."""
    import torch
    base = bank.tuning
    hmax = (bank.height + 15) // 16 * 16
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = {}
    for m in mults:
        bank.tuning = [min(s * m, hmax) if s else hmax for s in base]
        step()
        ts = []
        for _ in range(reps):
            start.record()
            step()
            stop.record()
            stop.synchronize()
            ts.append(start.elapsed_time(stop))
        times[m] = sorted(ts)[len(ts) // 2]
    m = min(times, key=times.get)
    bank.tuning = [min(s * m, hmax) if s else hmax for s in base]
    return {"seg_rows": bank.tuning, "candidates_ms": {f"x{mm}": round(t, 4) for mm, t in times.items()}}
