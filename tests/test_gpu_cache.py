"""GPU: the inference cache (the slice's direction-independent part, built
once per Gaussian) and the render-only forward that reads it, through the C
ABI: the cache against the oracle's, the images against the full forward."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2410_04974_amd import SixDGSError, build_cache
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def test_cache_matches_oracle():
    w, pn = G.scene("c2", 5000)
    cache = build_cache(G.to_dev(pn)).cpu().numpy().astype(np.float64)
    ref = oracle.static_part(pn)
    for nm, (a, b) in {"sigma_cond": (0, 6), "K": (6, 15), "sigma_d_inv": (15, 21), "alpha": (21, 22)}.items():
        err = np.linalg.norm(cache[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b])
        print("cache", nm, "rel err", err, flush=True)
        assert err < 1e-5


@pytest.mark.parametrize("tile", [(16, 16), (8, 32)])
def test_cached_forward_equals_forward(tile):
    w, pn = G.scene("c3", 30000)
    cams = synth.fibonacci_cameras(3, [(320, 240), (200, 200), (128, 300)])
    r = G.renderer(tile=tile)
    p = G.to_dev(pn)
    full = [im.clone() for im in r.forward(p, cams)]
    cache = build_cache(p)
    cached = r.forward_cached(p, cache, cams)
    torch.cuda.synchronize()
    for a, b in zip(full, cached):
        assert torch.equal(a, b)  # the same float operations on the same values


def test_cached_forward_matches_oracle():
    w, pn = G.scene("c1", 20000)
    cam = synth.default_camera(256, 192)
    env = oracle.render_envelope(pn, cam)
    r = G.renderer()
    p = G.to_dev(pn)
    img = r.forward_cached(p, build_cache(p), [cam])[0].cpu().numpy().astype(np.float64)
    G.check_envelope(img, None, env, "cached forward")


def test_no_backward_after_cached_forward():
    w, pn = G.scene("c1", 2000)
    cam = synth.default_camera(64, 64)
    r = G.renderer()
    p = G.to_dev(pn)
    r.forward_cached(p, build_cache(p), [cam])
    with pytest.raises(SixDGSError):
        r.backward(p, [torch.zeros((3, 64, 64), device=G.DEV)])
    lam = torch.zeros(pn.shape[1], device=G.DEV)
    r.ctx.set_lambda(lam, None)
    with pytest.raises(SixDGSError):
        r.forward_cached(p, build_cache(p), [cam])
