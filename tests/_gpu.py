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


# ------------------------------------------------------------- pixel parity
PIX_TOL = 1e-4  # absolute bar on colour and final transmittance


def _env_pixels(a):
    """An oracle output for a full frame ([3, H, W] / [H, W]) or a pixel list
    ([npix, 3] / [npix]) as [npix, 3] / [npix]."""
    a = np.asarray(a)
    if a.ndim == 3:
        return a.reshape(a.shape[0], -1).T
    return a.reshape(a.shape[0], -1) if a.ndim == 2 and a.shape[1] == 3 else a.reshape(-1)


def check_envelope(img, T, env, tag, say=print):
    """Every pixel of the GPU image (colour and, when T is given, final
    transmittance) lies inside the oracle's decision envelope up to PIX_TOL;
    on pixels with one decision path that is the definition's value itself.
    img: [3, H, W] or [3, npix] (T: [H, W] or [npix]); env: the
    oracle.render_envelope output for the same pixels.  Returns the statistics it prints."""
    c = np.asarray(img, np.float64).reshape(3, -1).T
    lo, hi, nom = _env_pixels(env["lo"]), _env_pixels(env["hi"]), _env_pixels(env["color"])
    amb = _env_pixels(env["ambiguous"]).astype(bool)
    out = np.maximum(lo - c, c - hi).max(axis=1)
    if T is not None:
        t = np.asarray(T, np.float64).reshape(-1)
        out = np.maximum(out, np.maximum(_env_pixels(env["T_lo"]) - t, t - _env_pixels(env["T_hi"])))
    err = np.abs(c - nom).max(axis=1)
    width = (hi - lo).max(axis=1)
    st = {"pixels": len(c), "max_outside": float(out.max()), "max_err_unambiguous": float(err[~amb].max()) if (~amb).any() else 0.0,
          "ambiguous_frac": float(amb.mean()), "width_gt_tol_frac": float((width > PIX_TOL).mean()),
          "max_err_to_definition": float(err.max())}
    say(tag, {k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in st.items()})
    assert not _env_pixels(env["unresolved"]).astype(bool).any()
    assert env["near_z"] == 0
    assert st["max_outside"] <= PIX_TOL, st
    return st


def grad_mask(env):
    """Pixels whose upstream gradient a gradient comparison must zero: those
    with any threshold decision a float32 renderer may take the other way
    (the gradient there depends on which way it goes)."""
    return env["flags"] != 0
