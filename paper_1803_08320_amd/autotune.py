"""Launch-shape autotuner for the integrate and camera kernels.

Times each candidate launch shape on a sample of the real work (HIP events on the
current stream) and keeps the fastest.  Results are cached per (device,
operation, precision, size bucket) in a JSON file: $MALBEC_TUNE_CACHE, else
_build/autotune.json next to the library.  Launch shape never changes results
(every lane's arithmetic is independent of the grid), only speed.
"""
from __future__ import annotations

import json
import os
import threading

import torch

from . import (Camera, _HERE, integrate, new_lane_arrays, trace_camera)

_lock = threading.Lock()
BLOCKS = (64, 128, 192, 256)
CHUNKS = (8, 32, 128)


def _cache_path():
    return os.environ.get("MALBEC_TUNE_CACHE", os.path.join(_HERE, "_build", "autotune.json"))


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = _cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _key(*parts):
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "|".join([getattr(dev, "gcnArchName", dev.name)] + [str(p) for p in parts])


def _bucket(n):
    return 1 << max(0, int(n - 1).bit_length())


def _time(fn, reps=2):
    fn()  # warm-up
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        a.record()
        fn()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def integrate_block(state, spacetimes, h, precision="f64", probe_steps=200, max_lanes=1 << 18,
                    refresh=False, **kw):
    """Best threads-per-block for malbec_integrate on this batch (cached)."""
    n = state.shape[-1]
    key = _key("integrate", precision, _bucket(n), len(spacetimes) if isinstance(spacetimes, list) else 1)
    with _lock:
        cache = _load()
        if key in cache and not refresh:
            return cache[key]["block"]
    m = min(n, max_lanes)
    sample = state[:, :m].contiguous()
    work = torch.empty_like(sample)
    status, steps = new_lane_arrays(m, device=state.device)
    times = {}
    for blk in BLOCKS:
        def run():
            work.copy_(sample)
            status.zero_()
            steps.zero_()
            integrate(work, status, steps, spacetimes, h=h, n_steps=probe_steps, precision=precision,
                      block=blk, **kw)
        times[blk] = _time(run)
    best = min(times, key=times.get)
    with _lock:
        cache = _load()
        cache[key] = {"block": best, "ms": times}
        _store(cache)
    return best


def camera_shape(cam: Camera, sample=256, refresh=False):
    """Best (block, steps_per_chunk) for the persistent camera kernel (cached), timed on a
    sample x sample image of the same camera."""
    key = _key("camera", _bucket(cam.nx * cam.ny), cam.a, cam.max_steps)
    with _lock:
        cache = _load()
        if key in cache and not refresh:
            return tuple(cache[key]["shape"])
    small = Camera(**{**cam.__dict__, "nx": min(sample, cam.nx), "ny": min(sample, cam.ny),
                      "persistent": 1})
    times = {}
    for blk in BLOCKS:
        for ch in CHUNKS:
            c = Camera(**{**small.__dict__, "block": blk, "steps_per_chunk": ch})
            times[(blk, ch)] = _time(lambda: trace_camera(c), reps=1)
    best = min(times, key=times.get)
    with _lock:
        cache = _load()
        cache[key] = {"shape": list(best), "ms": {"%d,%d" % k: v for k, v in times.items()}}
        _store(cache)
    return best
