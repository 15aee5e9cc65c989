"""Tile shape and LDS batch-depth autotuner.

The image does not depend on either setting (the per-pixel arithmetic and the
per-pixel Gaussian order are the same for every tile shape), so the tuner is
free to pick the fastest.  It times a forward + backward of the caller's own
workload for each candidate on the current stream with HIP events, and caches
the winner in a JSON file keyed by device and workload shape.
"""
from __future__ import annotations

import json
import os

import torch

from .render import Renderer

CANDIDATES = [((16, 16), 256), ((16, 16), 128), ((32, 8), 256), ((32, 8), 128), ((8, 32), 256), ((8, 32), 128)]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sixdgs_autotune.json")


def _key(n, cams):
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{dev}|n={n}|views=" + ",".join(f"{c.width}x{c.height}" for c in cams)


def _time_config(params, cams, dls, tile, batch, iters):
    r = Renderer(tile=tile, batch=batch)
    r.forward(params, cams)
    torch.cuda.synchronize()
    r.configure(pair_capacity=int(r.ctx.sizes()["pairs"] * 1.3) + 4096)
    g = torch.empty_like(params)
    for _ in range(2):
        r.forward(params, cams)
        r.backward(params, dls, grad=g)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        r.forward(params, cams)
        r.backward(params, dls, grad=g)
    e1.record()
    torch.cuda.synchronize()
    r.ctx.check()
    return e0.elapsed_time(e1) / iters


def autotune(params, cams, candidates=CANDIDATES, iters=5, cache=DEFAULT_CACHE, use_cache=True):
    """Returns {"tile": (w, h), "batch": b, "ms": t, "timings": {...}} for the
    fastest forward + backward of ``params`` over ``cams``."""
    key = _key(params.shape[1], cams)
    if use_cache and cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                hit = json.load(f).get(key)
            if hit:
                hit["tile"] = tuple(hit["tile"])
                return hit
        except (OSError, ValueError):
            pass
    gen = torch.Generator(device=params.device).manual_seed(0)
    dls = [torch.randn((3, c.height, c.width), device=params.device, generator=gen) for c in cams]
    timings = {}
    for tile, batch in candidates:
        timings[f"{tile[0]}x{tile[1]}/{batch}"] = _time_config(params, cams, dls, tile, batch, iters)
    best = min(timings, key=timings.get)
    tw, rest = best.split("x")
    th, b = rest.split("/")
    res = {"tile": (int(tw), int(th)), "batch": int(b), "ms": timings[best], "timings": timings}
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data[key] = dict(res, tile=list(res["tile"]))
            with open(cache, "w") as f:
                json.dump(data, f, indent=1)
        except (OSError, ValueError):
            pass
    return res
