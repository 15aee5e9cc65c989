"""Helpers for the GPU tests: running the HIP path through its C ABI on
seeded inputs and turning results into numpy."""
from __future__ import annotations

import numpy as np
import torch

import synth

DEV = "cuda:0"


def renderer(**kw):
    from paper_2410_04974_amd import Renderer
    return Renderer(**kw)


def to_dev(params: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).to(DEV)


def render(params, cams, **kw):
    """Forward on the GPU; returns (renderer, params tensor, [images as numpy])."""
    r = renderer(**kw)
    p = to_dev(params)
    imgs = r.forward(p, cams)
    torch.cuda.synchronize()
    return r, p, [im.cpu().numpy().astype(np.float64) for im in imgs]


def records(r):
    from paper_2410_04974_amd import _lib
    rec = r.ctx.export(_lib.EXPORT_RECORDS)
    tiles = r.ctx.export(_lib.EXPORT_TILES)
    return rec, tiles


REC_U, REC_V, REC_QXX, REC_QXY, REC_QYY, REC_AC, REC_EX, REC_EY, REC_R, REC_G, REC_B, REC_DEPTH = range(12)


def scene(name, n=None):
    w = synth.workload(name, n_override=n)
    return w, synth.make_scene(w.scene)


def rel_err(a, b, floor):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)
