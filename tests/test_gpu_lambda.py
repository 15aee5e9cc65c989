"""GPU: the learnable per-Gaussian lambda (sigmoid of a raw value per
Gaussian, in place of the scalar setting) through the C ABI, against the
oracle; its Adam; training with it."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def _group_errors(g, ref):
    out = {}
    for nm, (a, b) in {"mu_p": (0, 3), "mu_d": (3, 6), "L": (6, 27), "sh": (27, 75), "opacity": (75, 76)}.items():
        out[nm] = np.linalg.norm(g[a:b] - ref[a:b]) / max(np.linalg.norm(ref[a:b]), 1e-30)
    return out


def test_lambda_array_matches_oracle_forward_and_backward():
    w, pn = G.scene("c1", 20000)
    cam = synth.default_camera(256, 256)
    raw = np.random.default_rng(21).normal(0.0, 1.5, pn.shape[1]).astype(np.float32)
    env = oracle.render_envelope(pn, cam, lambda_raw=raw)
    r = G.renderer()
    p = G.to_dev(pn)
    lam = torch.from_numpy(raw).to(G.DEV)
    glam = torch.full_like(lam, float("nan"))
    r.ctx.set_lambda(lam, glam)
    img = r.forward(p, [cam])[0].cpu().numpy()
    G.check_envelope(img, None, env, "lambda array")
    dl = synth.upstream_gradient([cam])[0].astype(np.float64)
    dl[:, G.grad_mask(env)] = 0.0
    g = r.backward(p, [torch.from_numpy(dl.astype(np.float32)).to(G.DEV)]).cpu().numpy().astype(np.float64)
    ref, _, ref_lam = oracle.backward(pn, cam, dl, lambda_raw=raw)
    errs = _group_errors(g, ref)
    gl = glam.cpu().numpy().astype(np.float64)
    errs["lambda"] = np.linalg.norm(gl - ref_lam) / np.linalg.norm(ref_lam)
    print("lambda array: grad rel err per group", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert np.isfinite(gl).all()
    assert all(v < 1e-3 for v in errs.values())


def test_constant_lambda_array_equals_scalar_setting():
    w, pn = G.scene("c1", 20000)
    cam = synth.default_camera(200, 160)
    p = G.to_dev(pn)
    r0 = G.renderer(lambda_opa=0.35)
    img0 = r0.forward(p, [cam])[0]
    r1 = G.renderer(lambda_opa=0.9)  # the scalar must be ignored while the array is attached
    lam = torch.full((pn.shape[1],), math.log(0.35 / 0.65), device=G.DEV)
    r1.ctx.set_lambda(lam, None)
    img1 = r1.forward(p, [cam])[0]
    torch.cuda.synchronize()
    assert float((img0 - img1).abs().max()) < 1e-5  # sigmoid(logit(0.35)) rounds to 0.35 within an ulp or two
    r1.ctx.set_lambda(None, None)
    img2 = r1.forward(p, [cam])[0]
    assert float((img2 - r0.forward(p, [cam])[0]).abs().max()) > 1e-3  # back to the scalar 0.9


def test_adam_vec_matches_oracle():
    from paper_2410_04974_amd import _lib
    n = 1001
    rng = np.random.default_rng(8)
    p0 = rng.normal(size=n).astype(np.float32)
    pd = torch.from_numpy(p0).to(G.DEV)
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    counter = torch.zeros(1, dtype=torch.int32, device=G.DEV)
    lr = 1e-2
    ref_p, ref_m, ref_v = p0.astype(np.float64)[None], np.zeros((1, n)), np.zeros((1, n))
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        _lib.adam_vec(pd, torch.from_numpy(g).to(G.DEV), md, vd, lr, step_counter=counter)
        counter += 1
        f = lambda x: float(np.float32(x))
        ref_p, ref_m, ref_v = oracle.adam_step(ref_p, g[None].astype(np.float64), ref_m, ref_v, step, [f(lr)] * 6,
                                               b1=f(0.9), b2=f(0.999), eps=f(1e-15))
    torch.cuda.synchronize()
    assert np.allclose(pd.cpu().numpy(), ref_p[0], rtol=1e-5, atol=1e-6)
    assert np.allclose(md.cpu().numpy(), ref_m[0], rtol=1e-5, atol=1e-7)


def test_training_with_learnable_lambda():
    """Steps with a learnable lambda move it and lower the loss; with
    train_lambda off it stays fixed while the other parameters still train."""
    from paper_2410_04974_amd import Renderer, Trainer
    w, pn = G.scene("c2", 20000)
    cam = synth.default_camera(200, 160)
    tgt = Renderer().forward(torch.from_numpy(synth.perturbed(pn)).to(G.DEV), [cam])
    lam = torch.full((pn.shape[1],), math.log(0.35 / 0.65), device=G.DEV)
    tr = Trainer(G.to_dev(pn), Renderer(), lambda_raw=lam)
    losses = [float(tr.step([cam], tgt)) for _ in range(20)]
    torch.cuda.synchronize()
    moved = float((tr.lambda_raw - math.log(0.35 / 0.65)).abs().max())
    print("lambda moved by", moved, "loss", losses[0], "->", losses[-1], flush=True)
    assert moved > 1e-3 and losses[-1] < losses[0]
    assert torch.isfinite(tr.grad_lambda).all()
    tr.train_lambda = False
    before = tr.lambda_raw.clone()
    p_before = tr.params.clone()
    tr.step([cam], tgt)
    torch.cuda.synchronize()
    assert torch.equal(before, tr.lambda_raw) and not torch.equal(p_before, tr.params)
