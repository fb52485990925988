"""In-project autotuner for the batch launch variants.

``tune(op, run, key)`` times every variant of ``op`` ("das_batch" or
"apply_batch") by calling ``run(variant)`` under HIP events on the current
stream, keeps the fastest, and records it in a JSON cache (path from the
``TIDAS_TUNE_CACHE`` environment variable, default
``~/.cache/tidas/tune.json``) keyed by the device name, the op and a
caller-supplied shape-class key.  Variants only change launch shapes and
pipelining depth, never the arithmetic: every variant returns identical
results, so tuning cannot change an output.
"""
import json
import os
import threading

import torch

from . import _lib

N_VARIANTS = {"das_batch": _lib.DAS_BATCH_VARIANTS, "apply_batch": _lib.APPLY_BATCH_VARIANTS}
_lock = threading.Lock()


def cache_path():
    return os.environ.get("TIDAS_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "tidas", "tune.json"))


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(tab):
    path = cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _full_key(op, key):
    return f"{torch.cuda.get_device_name()}|{op}|{key}"


def lookup(op, key):
    """Cached variant for (device, op, key) or None."""
    with _lock:
        rec = _load().get(_full_key(op, key))
    return None if rec is None else int(rec["variant"])


def time_variant(run, variant, reps=3, warmup=1):
    for _ in range(warmup):
        run(variant)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run(variant)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(op, run, key, reps=3, force=False):
    """Best variant of ``op`` for ``run``; cached under ``key`` unless ``force``."""
    if not force:
        v = lookup(op, key)
        if v is not None:
            return v, None
    times = {v: time_variant(run, v, reps) for v in range(N_VARIANTS[op])}
    best = min(times, key=times.get)
    with _lock:
        tab = _load()
        tab[_full_key(op, key)] = {"variant": best, "ms": times[best],
                                   "all_ms": {str(k): round(t, 6) for k, t in times.items()}}
        _store(tab)
    return best, times
