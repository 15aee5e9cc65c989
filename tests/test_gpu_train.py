"""GPU parity of the training-step pieces: L1 loss, Adam, and the fused
backward + Adam path, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests import _gpu as G

pytestmark = pytest.mark.gpu

LR = (1.6e-4, 1e-3, 1e-2, 2.5e-3, 1.25e-4, 5e-2)


def test_l1_loss_and_gradient_match_oracle():
    """Images of different sizes in one call (one grid row each, the large
    one capped at its block count and strided), then two small ones again."""
    rng = np.random.default_rng(4)
    shapes = [(3, 37, 53), (3, 64, 64), (3, 720, 1280)]
    imgs = [rng.random(s).astype(np.float32) for s in shapes]
    tgts = [rng.random(s).astype(np.float32) for s in shapes]
    tgts[1][0, :3, :3] = imgs[1][0, :3, :3]  # exact ties: zero gradient
    r = G.renderer()
    for sel in ([0, 2, 1], [0, 1]):
        im = [imgs[k] for k in sel]
        tg = [tgts[k] for k in sel]
        di = [torch.from_numpy(a).to(G.DEV) for a in im]
        dt = [torch.from_numpy(a).to(G.DEV) for a in tg]
        dl = [torch.empty_like(a) for a in di]
        loss = torch.zeros(1, device=G.DEV)
        r.ctx.l1_loss(di, dt, dl, loss)
        ref_loss, ref_grads = oracle.l1_loss(im, tg)
        assert abs(float(loss) - ref_loss) <= 1e-6 * ref_loss, sel
        for g, rg in zip(dl, ref_grads):
            assert np.allclose(g.cpu().numpy(), rg, rtol=1e-6, atol=0)


@pytest.mark.parametrize("n", [1000, 1001])  # float4 and scalar kernels
def test_adam_matches_oracle_over_steps(n):
    from paper_2410_04974_amd import adam
    rng = np.random.default_rng(5)
    p = rng.normal(size=(76, n)).astype(np.float32)
    pd = torch.from_numpy(p).to(G.DEV)
    md = torch.zeros_like(pd)
    vd = torch.zeros_like(pd)
    ref_p, ref_m, ref_v = p.astype(np.float64), np.zeros((76, n)), np.zeros((76, n))
    for step in range(1, 5):
        g = rng.normal(size=(76, n)).astype(np.float32)
        adam(pd, torch.from_numpy(g).to(G.DEV), md, vd, LR, step)
        # the hyper-parameters the GPU receives are float32 (1 - float32(0.999) is 1.3e-5 off 0.001)
        ref_p, ref_m, ref_v = oracle.adam_step(ref_p, g, ref_m, ref_v, step, [float(np.float32(x)) for x in LR],
                                               b1=float(np.float32(0.9)), b2=float(np.float32(0.999)),
                                               eps=float(np.float32(1e-15)))
    torch.cuda.synchronize()
    assert np.allclose(pd.cpu().numpy(), ref_p, rtol=1e-5, atol=1e-6)
    assert np.allclose(md.cpu().numpy(), ref_m, rtol=1e-5, atol=1e-7)
    assert np.allclose(vd.cpu().numpy(), ref_v, rtol=1e-5, atol=1e-9)


@pytest.mark.parametrize("case", ["one_view", "three_views_lambda", "three_views_rgb"])
def test_fused_backward_adam_equals_backward_then_adam(case):
    """Adam inside the chain rule's kernel (the training default) against the
    gradient written out and the streaming Adam kernel, over three steps.  With
    several views the fused kernel sums the colour rows in LDS and reads the
    coefficients per view; a learnable lambda shares the step's count; the
    densification statistics are accumulated by both."""
    from paper_2410_04974_amd import Renderer, Trainer
    w, pn = G.scene("c2", 20000)
    if case == "one_view":
        cams = [synth.default_camera(200, 160)]
    else:
        cams = [synth.default_camera(200, 160), synth.default_camera(97, 61), synth.default_camera(64, 150)]
    rgb = case == "three_views_rgb"
    tgt = Renderer(rgb_color=rgb).forward(torch.from_numpy(synth.perturbed(pn)).to(G.DEV), cams)
    tgt = [t.clone() for t in tgt]
    outs = []
    for fused in (True, False):
        p = torch.from_numpy(pn).to(G.DEV)
        lam = None
        if case == "three_views_lambda":
            lam = torch.from_numpy(np.random.default_rng(7).normal(0.0, 0.5, pn.shape[1]).astype(np.float32)).to(G.DEV)
        tr = Trainer(p, Renderer(rgb_color=rgb), lambda_raw=lam)
        dens = torch.zeros((2, pn.shape[1]), device=G.DEV)
        for _ in range(3):
            tr.step(cams, tgt, densify=dens, fused=fused)
        torch.cuda.synchronize()
        assert int(tr.step_counter.item()) == 3
        o = [tr.params.cpu().numpy(), tr.m.cpu().numpy(), tr.v.cpu().numpy(), dens.cpu().numpy()]
        if lam is not None:
            o.append(tr.lambda_raw.cpu().numpy())
        outs.append(o)
    for a, b in zip(outs[0], outs[1]):
        # The two paths differ in the order of the backward's float atomics (and
        # in where Adam's bias correction is formed).  Adam's update is close to
        # lr * sign(g) early on, so a gradient at the rounding-noise level may
        # move the other way: allow a small fraction of such elements (more of
        # them with short backward chunks, whose partial sums are more).
        close = np.isclose(a, b, rtol=1e-4, atol=1e-6 * max(1.0, np.abs(b).max()))
        assert close.mean() > 1 - 1e-3, close.mean()
    assert not np.array_equal(outs[0][0], pn)  # the parameters moved


@pytest.mark.parametrize("views", [1, 3, "two_1080p"])
def test_forward_with_l1_equals_forward_then_l1(views):
    """The L1 loss formed as the forward writes the pixels: the same images and
    dL/dI bit for bit as a forward followed by sixdgs_l1_loss, the same loss up
    to the order of the sum, and the same backward state."""
    from paper_2410_04974_amd import Renderer, _lib
    w, pn = G.scene("c2", 20000)
    if views == "two_1080p":  # 16,200 tiles: the loss is summed in two levels
        cams = [synth.default_camera(1920, 1080), synth.default_camera(1920, 1080)]
    else:
        cams = [synth.default_camera(160, 128), synth.default_camera(97, 61), synth.default_camera(40, 200)][:views]
    p = torch.from_numpy(pn).to(G.DEV)
    tgt = Renderer().forward(torch.from_numpy(synth.perturbed(pn)).to(G.DEV), cams)
    tgt = [t.clone() for t in tgt]
    out = []
    for fused in (False, True):
        r = Renderer()
        dl = [torch.full_like(t, 5.0) for t in tgt]
        loss = torch.full((1,), -1.0, device=G.DEV)
        if fused:
            imgs = r.forward(p, cams, targets=tgt, dl_dimages=dl, loss=loss)
        else:
            imgs = r.forward(p, cams)
            r.ctx.l1_loss(imgs, tgt, dl, loss)
        T = r.ctx.export(_lib.EXPORT_T_FINAL)
        g = r.backward(p, dl)
        torch.cuda.synchronize()
        out.append(([i.clone() for i in imgs], [d.clone() for d in dl], float(loss.item()), T, g.clone()))
    (i0, d0, l0, T0, g0), (i1, d1, l1, T1, g1) = out
    assert all(torch.equal(a, b) for a, b in zip(i0, i1))
    assert all(torch.equal(a, b) for a, b in zip(d0, d1))
    assert np.array_equal(T0, T1)
    assert l1 > 0 and abs(l1 - l0) <= 1e-5 * l0
    assert torch.allclose(g0, g1, rtol=1e-5, atol=1e-6 * float(g0.abs().max()))
    # an incomplete request is refused before any launch
    r = Renderer()
    with pytest.raises(ValueError):
        r.forward(p, cams, targets=tgt, loss=torch.zeros(1, device=G.DEV))


def test_fused_step_count_on_the_device_matches_the_host_count():
    """The fused backward + Adam with the step on the device (the training
    default) against the same kernel given the host's step count: the
    counter reads 3 after three steps, and the states agree."""
    from paper_2410_04974_amd import Renderer, Trainer
    w, pn = G.scene("c2", 20000)
    cam = synth.default_camera(160, 128)
    tgt = Renderer().forward(torch.from_numpy(synth.perturbed(pn)).to(G.DEV), [cam])
    tr = Trainer(torch.from_numpy(pn).to(G.DEV), Renderer())
    for _ in range(3):
        tr.step([cam], tgt)
    torch.cuda.synchronize()
    assert int(tr.step_counter.item()) == 3 and tr.step_count == 3
    # the host-count path of the same kernel, driven by hand
    r = Renderer()
    p = torch.from_numpy(pn).to(G.DEV)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    loss = torch.zeros(1, device=G.DEV)
    img = [torch.empty(3, cam.height, cam.width, device=G.DEV)]
    dl = [torch.empty_like(img[0])]
    for k in range(3):
        r.forward(p, [cam], out=img)
        r.ctx.l1_loss(img, tgt, dl, loss)
        r.ctx.backward_adam(p, dl, m, v, tr.lr, k + 1)
    torch.cuda.synchronize()
    for a, b in ((tr.params, p), (tr.m, m), (tr.v, v)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        close = np.isclose(a, b, rtol=1e-4, atol=1e-6 * max(1.0, np.abs(b).max()))
        assert close.mean() > 1 - 1e-3, close.mean()
    # advance = 0 leaves the counter to the caller
    r.forward(p, [cam], out=img)
    r.ctx.l1_loss(img, tgt, dl, loss)
    cnt = torch.full((1,), 7, device=G.DEV, dtype=torch.int32)
    r.ctx.backward_adam(p, dl, m, v, tr.lr, step_counter=cnt, advance=False)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 7


def test_densify_statistics_match_oracle():
    w, pn = G.scene("c1", 15000)
    cams = [synth.default_camera(160, 128), synth.look_at_camera((0.0, -4.0, 1.0), 96, 80)]
    from paper_2410_04974_amd import Renderer
    r = Renderer()
    p = G.to_dev(pn)
    r.forward(p, cams)
    dls = synth.upstream_gradient(cams)
    ambs = []
    for c, dl in zip(cams, dls):
        amb = G.grad_mask(oracle.render_envelope(pn, c))
        dl[:, amb] = 0.0
        ambs.append(amb)
    dens = torch.zeros((2, pn.shape[1]), device=G.DEV)
    r.backward(p, [torch.from_numpy(d).to(G.DEV) for d in dls], densify=dens)
    # visibility from the oracle's own records: alive and covering at least one tile
    vis = []
    for c in cams:
        o = oracle.preprocess(pn, c)
        b = oracle.bin_records(o["u"].astype(np.float32), o["v"].astype(np.float32), o["ex"].astype(np.float32),
                               o["ey"].astype(np.float32), o["depth"].astype(np.float32), o["alive"],
                               pn.shape[1], [c], 16, 16)
        vis.append(b["tiles_touched"] > 0)
    g2ds = [oracle.backward(pn, c, d.astype(np.float64))[1] for c, d in zip(cams, dls)]
    acc, cnt = oracle.densify_stats(g2ds, vis, cams)
    got = dens.cpu().numpy()
    same = got[1] == cnt  # a float32 extent may land on the other side of a tile edge
    assert same.mean() > 0.999
    assert np.allclose(got[0][same], acc[same], rtol=1e-3, atol=1e-4 * acc.max())


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_l1_dssim_loss_and_gradient_match_oracle(lam):
    """The full 3DGS loss over views of ragged sizes (tiles with partial edges,
    a view smaller than the window), value and dL/dI against the oracle."""
    rng = np.random.default_rng(12)
    shapes = [(3, 37, 53), (3, 64, 64), (3, 7, 9)]
    imgs = [rng.random(s).astype(np.float32) for s in shapes]
    tgts = [np.clip(a + rng.normal(0, 0.1, a.shape), 0, 1).astype(np.float32) for a in imgs]
    r = G.renderer()
    di = [torch.from_numpy(a).to(G.DEV) for a in imgs]
    dt = [torch.from_numpy(a).to(G.DEV) for a in tgts]
    dl = [torch.empty_like(a) for a in di]
    loss = torch.zeros(1, device=G.DEV)
    r.ctx.l1_dssim_loss(di, dt, dl, loss, lambda_dssim=lam)
    ref_loss, ref_grads = oracle.l1_dssim_loss(imgs, tgts, lam=lam)
    print("l1+dssim", float(loss), ref_loss, flush=True)
    assert abs(float(loss) - ref_loss) <= 1e-5 * ref_loss
    for g, rg in zip(dl, ref_grads):
        g = g.cpu().numpy()
        assert np.abs(g - rg).max() <= 1e-4 * np.abs(rg).max()


def test_training_with_dssim_lowers_the_loss():
    from paper_2410_04974_amd import Renderer, Trainer
    w, pn = G.scene("c2", 20000)
    cam = synth.default_camera(200, 160)
    tgt = Renderer().forward(torch.from_numpy(synth.perturbed(pn)).to(G.DEV), [cam])
    tr = Trainer(G.to_dev(pn), Renderer(), lambda_dssim=0.2)
    losses = [float(tr.step([cam], tgt)) for _ in range(15)]
    print("l1+dssim training", losses[0], "->", losses[-1], flush=True)
    assert losses[-1] < 0.8 * losses[0]
