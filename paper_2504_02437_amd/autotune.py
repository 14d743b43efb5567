"""Autotuner of the rasterizer's launch shape.

Sweeps the screen tile (8, 16, 32), the LDS batch (128, 256, 512) and the
threads per tile workgroup over the caller's actual workload, timing whole
forward + backward iterations with HIP events, and caches the fastest shape
per (device, image size, Gaussian-count bucket, view count) in a JSON file.
Outputs do not depend on the shape (a pixel evaluates an entry only inside
the entry's pixel box), so tuning never changes results.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os

import torch

from . import raster as R

BATCHES = (128, 256, 512)
THREADS = {8: (64,), 16: (64, 128, 256), 32: (128, 256)}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gsmap",
                             "autotune.json")


def shapes(tiles=(8, 16, 32)):
    return [(t, b, n) for t in tiles for n in THREADS[t] for b in BATCHES]


def cache_key(cams, n_gaussians):
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", props.name)
    bucket = 2 ** max(0, int(math.ceil(math.log2(max(1, n_gaussians)))))
    c = cams[0]
    return f"{arch}|{c.width}x{c.height}|n<={bucket}|V={len(cams)}"


def _time_iteration(rast, params, grad, dL, reps):
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for i in range(reps + 1):
        if i == 1:
            ev[0].record()
        grad.data.zero_()
        rast.forward(params)
        rast.backward(params, dL, grad)
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / reps


def autotune(params, cams, base: R.Settings | None = None, reps=3,
             tiles=(8, 16, 32), cache_path=DEFAULT_CACHE, use_cache=True,
             key_capacity=None, log=None):
    """Returns (best Settings, {shape: ms}) for rendering `params` into
    `cams`.  `base` supplies the non-shape settings (background, cut-offs)."""
    base = base or R.Settings()
    key = cache_key(cams, params.n())
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        t, b, n = cache[key]["shape"]
        return (dataclasses.replace(base, tile=t, lds_batch=b, block_threads=n),
                {tuple(cache[key]["shape"]): cache[key]["ms"]})
    grad = params.zeros_like()
    V = len(cams)
    dL = torch.full((V, 3, cams[0].height, cams[0].width),
                    1.0 / (3 * cams[0].height * cams[0].width),
                    device=params.data.device)
    times = {}
    for tile in tiles:
        s0 = dataclasses.replace(base, tile=tile, lds_batch=256,
                                 emit_keys=False, block_threads=0)
        rast = R.Rasterizer(cams, params.capacity, s0,
                            key_capacity=key_capacity,
                            device=params.data.device)
        rast.fit_key_capacity(params)
        for (t, b, n) in shapes((tile,)):
            rast.settings = dataclasses.replace(s0, lds_batch=b,
                                                block_threads=n)
            ms = _time_iteration(rast, params, grad, dL, reps)
            if rast.status()[0]:
                raise RuntimeError("key capacity exceeded while autotuning")
            times[(t, b, n)] = ms
            if log:
                log(f"autotune: tile {t} batch {b} threads {n}: {ms:.3f} ms")
        del rast
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        cache[key] = {"shape": list(best), "ms": times[best]}
        with open(cache_path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(cache_path + ".tmp", cache_path)
    t, b, n = best
    return dataclasses.replace(base, tile=t, lds_batch=b, block_threads=n), times
