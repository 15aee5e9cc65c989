"""GPU gradients on the full 100k-Gaussian, 800x800 sphere workload against
FP64 central finite differences of the oracle's forward, on a seeded subset
of 64 alive Gaussians.

The upstream gradient dL/dI ~ N(0, 1) lives on a 64x64 window of the image
(zero elsewhere and on pixels where a threshold decision of the walk is
undecided in float32, the oracle's decision envelope), so a
perturbation of one Gaussian only changes the loss through the window pixels
inside that Gaussian's extent box; the oracle renders exactly those pixels,
brute force over all 100k Gaussians.  Each Gaussian gets 4 of its 76
parameter rows, cycling so that the 64 Gaussians cover every row.  The
oracle renders with the Gaussians whose extent boxes reach the window: the
others have alpha < 1/255 on every window pixel (the box property pinned in
the oracle's own tests), so this is the same function, evaluated faster.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from tests import _gpu as G

pytestmark = pytest.mark.gpu

WIN = (368, 368, 64, 64)  # x0, y0, width, height: the sphere's front surface


def test_gradient_matches_fp64_finite_differences_on_64_gaussians():
    w, pn = G.scene("c1")
    cam = w.cameras[0]
    W, H = cam.width, cam.height
    x0, y0, ww, wh = WIN
    jj, ii = np.mgrid[y0:y0 + wh, x0:x0 + ww]
    win = (jj * W + ii).reshape(-1)
    amb = G.grad_mask(oracle.render_envelope(pn, cam, pixels=win))
    rng = np.random.default_rng(synth.SEED_UPSTREAM)
    dl_win = rng.normal(size=(len(win), 3))
    dl_win[amb] = 0.0
    dl = np.zeros((3, H * W), np.float32)
    dl[:, win] = dl_win.T
    dl = dl.reshape(3, H, W)

    r, p, _ = G.render(pn, [cam])
    g = r.backward(p, [torch.from_numpy(dl).to(G.DEV)]).cpu().numpy().astype(np.float64)

    rec = oracle.preprocess(pn, cam)
    m = 2.0
    near = np.nonzero(rec["alive"] & (rec["u"] + rec["ex"] > x0 - m) & (rec["u"] - rec["ex"] < x0 + ww + m) &
                      (rec["v"] + rec["ey"] > y0 - m) & (rec["v"] - rec["ey"] < y0 + wh + m))[0]
    sub = pn[:, near].astype(np.float64)  # index order kept: same depth tie-breaks
    col_full, _, _ = oracle.render_plain(pn, cam, pixels=win)
    col_sub, _, _ = oracle.render_plain(sub, cam, pixels=win)
    assert np.abs(col_full - col_sub).max() < 1e-12  # the reduced scene is the same function on the window
    cand = np.nonzero(rec["alive"][near] & (rec["u"][near] + rec["ex"][near] > x0) &
                      (rec["u"][near] - rec["ex"][near] < x0 + ww) & (rec["v"][near] + rec["ey"][near] > y0) &
                      (rec["v"][near] - rec["ey"][near] < y0 + wh))[0]
    dl_map = {int(k): dl_win[i] for i, k in enumerate(win)}
    px = ii.reshape(-1) + 0.5
    py = jj.reshape(-1) + 0.5
    live = np.array([np.any(dl_map[int(k)] != 0) for k in win])

    def box_pixels(gi):
        """Window pixels with an upstream gradient inside the (slightly grown) extent box of Gaussian gi."""
        bx0, bx1 = rec["u"][gi] - rec["ex"][gi] - 2, rec["u"][gi] + rec["ex"][gi] + 2
        by0, by1 = rec["v"][gi] - rec["ey"][gi] - 2, rec["v"][gi] + rec["ey"][gi] + 2
        return win[live & (px >= bx0) & (px <= bx1) & (py >= by0) & (py <= by1)]

    # the subset is drawn from the Gaussians that reach a window pixel with an upstream gradient
    cand = np.array([si for si in cand if len(box_pixels(near[si])) > 0])
    pick = np.sort(np.random.default_rng(synth.SEED_FD_SUBSET).choice(cand, 64, replace=False))

    def local_loss(params, pixels):
        col, _, _ = oracle.render_plain(params, cam, pixels=pixels)
        return float(sum((col[k] * dl_map[int(px)]).sum() for k, px in enumerate(pixels)))

    fd, an, rows_used = [], [], []
    discarded = 0
    for k, si in enumerate(pick):
        gi = near[si]  # index in the full scene
        sel = box_pixels(gi)
        for j in range(4):
            row = (4 * k + j) % 76
            base = float(sub[row, si])
            h = 1e-6 * max(1.0, abs(base))
            est = []
            for hh in (h, h / 2):
                pp = sub.copy()
                pp[row, si] = base + hh
                lp = local_loss(pp, sel)
                pp[row, si] = base - hh
                lm = local_loss(pp, sel)
                est.append((lp - lm) / (2 * hh))
            if abs(est[0] - est[1]) > 0.1 * max(abs(est[1]), 1e-6):
                discarded += 1  # a threshold was crossed inside the step
                continue
            fd.append(est[1])
            an.append(g[row, gi])
            rows_used.append(row)
    fd, an = np.array(fd), np.array(an)
    print(f"FD-64: {len(fd)} parameters compared, {discarded} discarded, "
          f"{len(set(rows_used))} distinct rows", flush=True)
    assert len(fd) >= 200
    scale = np.abs(fd).max()
    err = np.abs(an - fd)
    rel = np.linalg.norm(an - fd) / np.linalg.norm(fd)
    print(f"FD-64: max |g - fd| / max|fd| = {err.max() / scale:.2e}, norm rel err = {rel:.2e}", flush=True)
    # in norm, and per element relative to max(|fd|, 1e-2 max|fd|): a float32
    # gradient entry is a sum of many terms, so near-zero entries carry an
    # absolute error of order 1e-5 of the largest entry
    assert rel <= 1e-3
    assert np.all(err <= 1e-3 * np.maximum(np.abs(fd), 1e-2 * scale))
