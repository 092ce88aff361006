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
