"""GPU: the No-SH colour (the Sec. 5 ablation: a per-Gaussian RGB through a
sigmoid, held in the SH degree-0 rows) through the C ABI, against the oracle
in the same mode and against the SH colour with only degree-0 coefficients."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from tests import _gpu as G

pytestmark = pytest.mark.gpu

Y00 = 0.5 / math.sqrt(math.pi)


def _group_errors(g, ref):
    out = {}
    for nm, (a, b) in {"mu_p": (0, 3), "mu_d": (3, 6), "L": (6, 27), "rgb": (27, 30), "opacity": (75, 76)}.items():
        out[nm] = np.linalg.norm(g[a:b] - ref[a:b]) / max(np.linalg.norm(ref[a:b]), 1e-30)
    return out


def test_rgb_color_matches_oracle_forward_and_backward():
    w, pn = G.scene("c2", 20000)
    cam = synth.default_camera(256, 192)
    st = oracle.Settings(rgb_color=True)
    env = oracle.render_envelope(pn, cam, st)
    r, p, imgs = G.render(pn, [cam], rgb_color=True)
    G.check_envelope(imgs[0], None, env, "rgb colour")
    dl = synth.upstream_gradient([cam])[0].astype(np.float64)
    dl[:, G.grad_mask(env)] = 0.0
    g = r.backward(p, [torch.from_numpy(dl.astype(np.float32)).to(G.DEV)]).cpu().numpy().astype(np.float64)
    ref, _ = oracle.backward(pn, cam, dl, st)
    errs = _group_errors(g, ref)
    print("rgb colour: grad rel err per group", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert all(v < 1e-3 for v in errs.values())
    assert np.all(g[30:75] == 0.0)  # the unused SH rows


def test_rgb_color_equals_dc_only_sh_on_gpu():
    w, pn = G.scene("c1", 20000)
    cam = synth.default_camera(200, 160)
    c = np.random.default_rng(31).normal(0.0, 1.0, (3, pn.shape[1]))
    p_rgb = pn.copy()
    p_rgb[27:30] = c
    p_rgb[30:75] = 7.0  # ignored in this mode
    p_sh = pn.copy()
    p_sh[27:30] = c / Y00
    p_sh[30:75] = 0.0
    _, _, a = G.render(p_rgb, [cam], rgb_color=True)
    _, _, b = G.render(p_sh, [cam])
    d = float(np.abs(a[0] - b[0]).max())
    print("rgb vs dc-only sh: max image difference", d, flush=True)
    assert d < 1e-5  # the two colours differ only by float32 rounding of c / Y00 * Y00
    assert float(np.abs(a[0]).max()) > 0.05
