"""Tile shape, LDS batch-depth and backward-chunk autotuner.

The image does not depend on any of them (the per-pixel arithmetic and the
per-pixel Gaussian order are the same for every tile shape; the backward's
chunk only changes where its walks restart), so the tuner is free to pick the
fastest.  Short chunks spread the heavy tiles of a small frame over more
workgroups; with tens of thousands of tiles there is parallelism enough, and
longer chunks save the restarts.  It times a forward + backward of the caller's own
workload for each candidate on the current stream with HIP events, and caches
the winner in a JSON file keyed by device and workload shape.
"""
from __future__ import annotations

import json
import os

import torch

from .render import Renderer

# (tile, LDS batch depth, backward chunk); a batch longer than the chunk is cut to it
CANDIDATES = [(tile, batch, chunk) for tile in ((16, 16), (32, 8), (8, 32))
              for batch, chunk in ((256, 512), (256, 256), (128, 128), (64, 64))]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sixdgs_autotune.json")


def _key(n, cams):
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{dev}|n={n}|views=" + ",".join(f"{c.width}x{c.height}" for c in cams)


def _time_config(params, cams, dls, tile, batch, chunk, iters):
    r = Renderer(tile=tile, batch=batch, chunk=chunk)
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
    """Returns {"tile": (w, h), "batch": b, "chunk": c, "ms": t, "timings": {...}}
    for the fastest forward + backward of ``params`` over ``cams``."""
    key = _key(params.shape[1], cams)
    if use_cache and cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                hit = json.load(f).get(key)
            if hit and "chunk" in hit:
                hit["tile"] = tuple(hit["tile"])
                return hit
        except (OSError, ValueError):
            pass
    gen = torch.Generator(device=params.device).manual_seed(0)
    dls = [torch.randn((3, c.height, c.width), device=params.device, generator=gen) for c in cams]
    timings = {}
    for tile, batch, chunk in candidates:
        timings[f"{tile[0]}x{tile[1]}/{batch}/{chunk}"] = _time_config(params, cams, dls, tile, batch, chunk, iters)
    best = min(timings, key=timings.get)
    tw, rest = best.split("x")
    th, b, c = rest.split("/")
    res = {"tile": (int(tw), int(th)), "batch": int(b), "chunk": int(c), "ms": timings[best], "timings": timings}
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
