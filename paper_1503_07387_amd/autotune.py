"""Persistent cache of the autotuned decode tiling.

The library's autotuner (vbyte_autotune_decode / vbyte_autotune_batch in
include/vbyte.h) times every candidate tiling on the caller's workload and
applies the fastest.  This module keeps the winners in a JSON file keyed by
device name and a workload key, so later processes apply a stored tiling
without timing again:

    {"<device name>": {"<workload key>": {"segs_per_wave": 4,
                                          "waves_per_block": 8,
                                          "small_list_bytes": 16384,
                                          "tiles_per_chunk": 4,
                                          "ms": 0.118}}}

The default file is $VBYTE_TUNE_CACHE or ~/.cache/vbyte_tuning.json.
"""
import json
import os

import torch

from . import vbyte


def cache_path():
    return os.environ.get("VBYTE_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "vbyte_tuning.json"))


def _load(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path, d):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _bucket(x):
    """Power-of-two size class, so that similar workloads share an entry."""
    return int(x).bit_length()


def stream_key(nbytes, n, delta):
    return f"stream:delta={int(bool(delta))}:bytes=2^{_bucket(nbytes)}:ints=2^{_bucket(n)}"


def batch_key(nbytes, nlists, delta):
    return f"batch:delta={int(bool(delta))}:bytes=2^{_bucket(nbytes)}:lists=2^{_bucket(nlists)}"


def _apply(entry):
    vbyte.set_tuning(entry["segs_per_wave"], entry["waves_per_block"], entry["small_list_bytes"],
                     tiles_per_chunk=entry.get("tiles_per_chunk", 0))


def _tuned(key, run, path, retune):
    path = path or cache_path()
    dev = torch.cuda.get_device_name()
    d = _load(path)
    entry = d.get(dev, {}).get(key)
    if entry is not None and not retune:
        _apply(entry)
        return entry, None
    points = run()
    best = vbyte.get_tuning()
    ms = min((p["ms"] for p in points if all(p[k] == best[k] for k in best)), default=None)
    entry = dict(best, ms=ms)
    d.setdefault(dev, {})[key] = entry
    _store(path, d)
    return entry, points


def tune_stream(data, n, *, delta=False, path=None, retune=False, reps=5):
    """Apply the cached (or freshly timed) tiling for a single-stream decode
    of `data`.  Returns (entry, timed candidates or None on a cache hit)."""
    key = stream_key(data.numel(), n, delta)
    return _tuned(key, lambda: vbyte.autotune_decode(data, n, delta=delta, reps=reps), path, retune)


def tune_batch(data, byte_off, out_off, *, delta=False, path=None, retune=False, reps=3):
    """Same for a batched CSR decode (tiling and small-list threshold)."""
    key = batch_key(data.numel(), byte_off.numel() - 1, delta)
    return _tuned(key, lambda: vbyte.autotune_batch(data, byte_off, out_off, delta=delta,
                                                    reps=reps), path, retune)
