"""Launch-shape autotuner for the integrate and camera kernels.

Times each candidate launch shape on a sample of the real work (HIP events on the
current stream) and keeps the fastest: threads per block for malbec_integrate, plus
the retire/refill interval (steps_per_chunk) of its persistent work-queue kernel, and
(block, steps_per_chunk) of the persistent camera kernel.  Results are cached per
(device, operation, precision, formulation, persistent or not, number of spacetimes,
size bucket) in a JSON file: $MALBEC_TUNE_CACHE, else _build/autotune.json next to
the library.  The binding's integrate() and trace_camera() take a cached shape when
called with block = 0 (and, for persistent launches, steps_per_chunk = 0); without a
cached entry the library's defaults apply (256 threads per block; refill every 64
steps for integrate, every 32 for the camera).  Launch shape never changes results
(every lane's arithmetic is independent of the grid), only speed.
"""
from __future__ import annotations

import json
import os
import threading

import torch

from . import (Camera, _HERE, _spacetimes, integrate, new_lane_arrays, trace_camera)

_lock = threading.Lock()
BLOCKS = (64, 128, 192, 256)
CHUNKS = (8, 32, 128)
_mem = None  # the cache file's content, loaded once per process
_arch = {}


def _cache_path():
    return os.environ.get("MALBEC_TUNE_CACHE", os.path.join(_HERE, "_build", "autotune.json"))


def _load():
    global _mem
    if _mem is None or _mem[0] != _cache_path():
        try:
            with open(_cache_path()) as f:
                _mem = (_cache_path(), json.load(f))
        except (OSError, ValueError):
            _mem = (_cache_path(), {})
    return _mem[1]


def _store(cache):
    global _mem
    path = _cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    _mem = (path, cache)


def _key(*parts):
    d = torch.cuda.current_device()
    if d not in _arch:
        dev = torch.cuda.get_device_properties(d)
        _arch[d] = getattr(dev, "gcnArchName", dev.name)
    return "|".join([_arch[d]] + [str(p) for p in parts])


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


def _integrate_key(n, n_st, precision, formulation, persistent):
    return _key("integrate", precision, formulation, "persistent" if persistent else "plain",
                n_st, _bucket(n))


def lookup_integrate(n, n_st, precision="f64", formulation="christoffel", persistent=False):
    """The cached (block, steps_per_chunk) of an integrate launch, or None (no timing)."""
    with _lock:
        e = _load().get(_integrate_key(n, n_st, precision, formulation, persistent))
    return (e["block"], e["chunk"]) if e else None


def integrate_shape(state, spacetimes, h, precision="f64", formulation="christoffel",
                    persistent=False, st_of_lane=None, probe_steps=200, max_lanes=1 << 18,
                    refresh=False, **kw):
    """Best (block, steps_per_chunk) for malbec_integrate on this batch (cached).  For a
    plain launch the chunk is 0 (all steps in one launch); for the persistent kernel it
    is the retire/refill interval.  Timed on the first max_lanes lanes (with their
    spacetime indices) over probe_steps steps."""
    n = state.shape[-1]
    n_st = len(_spacetimes(spacetimes))
    key = _integrate_key(n, n_st, precision, formulation, persistent)
    with _lock:
        e = _load().get(key)
    if e and not refresh:
        return e["block"], e["chunk"]
    m = min(n, max_lanes)
    sample = state[:, :m].contiguous()
    sol = None if st_of_lane is None else st_of_lane[:m].contiguous()
    work = torch.empty_like(sample)
    status, steps = new_lane_arrays(m, device=state.device)
    times = {}
    for blk in BLOCKS:
        for ch in (CHUNKS if persistent else (0,)):
            def run():
                work.copy_(sample)
                status.zero_()
                steps.zero_()
                integrate(work, status, steps, spacetimes, h=h, n_steps=probe_steps,
                          precision=precision, formulation=formulation, persistent=persistent,
                          block=blk, steps_per_chunk=ch, st_of_lane=sol, **kw)
            times[(blk, ch)] = _time(run)
    best = min(times, key=times.get)
    with _lock:
        cache = dict(_load())
        cache[key] = {"block": best[0], "chunk": best[1],
                      "ms": {"%d,%d" % k: v for k, v in times.items()}}
        _store(cache)
    return best


def integrate_block(state, spacetimes, h, precision="f64", **kw):
    """Best threads per block for a plain integrate launch (integrate_shape's block)."""
    return integrate_shape(state, spacetimes, h, precision=precision, **kw)[0]


def _camera_key(cam: Camera):
    return _key("camera", _bucket(cam.nx * cam.ny), cam.a, cam.max_steps)


def lookup_camera(cam: Camera):
    """The cached (block, steps_per_chunk) of the persistent camera kernel, or None."""
    with _lock:
        e = _load().get(_camera_key(cam))
    return tuple(e["shape"]) if e else None


def camera_shape(cam: Camera, sample=1024, refresh=False):
    """Best (block, steps_per_chunk) for the persistent camera kernel (cached), timed on a
    sample x sample image of the same camera (the best of two launches after a warm-up).
    The default 1024 x 1024 sample fills the device several times over, as the full image
    does; on a 256 x 256 one (a single wave per SIMD, 2 ms launches) the choice between
    the shapes, a few per cent apart, followed the timing noise."""
    key = _camera_key(cam)
    with _lock:
        e = _load().get(key)
    if e and not refresh:
        return tuple(e["shape"])
    small = Camera(**{**cam.__dict__, "nx": min(sample, cam.nx), "ny": min(sample, cam.ny),
                      "persistent": 1})
    times = {}
    for blk in BLOCKS:
        for ch in CHUNKS:
            c = Camera(**{**small.__dict__, "block": blk, "steps_per_chunk": ch})
            times[(blk, ch)] = _time(lambda: trace_camera(c), reps=2)
    best = min(times, key=times.get)
    with _lock:
        cache = dict(_load())
        cache[key] = {"shape": list(best), "ms": {"%d,%d" % k: v for k, v in times.items()}}
        _store(cache)
    return best
