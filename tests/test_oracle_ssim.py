"""Pins of the oracle's SSIM term (CPU only): closed forms, the maximum at
identical images, an independent direct evaluation, and FP64 finite
differences of the hand-written gradient."""
import numpy as np

import oracle
from oracle import dssim as S


def test_window_is_the_normalised_gaussian():
    w = S.window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-14
    assert abs(w[5, 6] / w[5, 5] - np.exp(-1 / (2 * 1.5 ** 2))) < 1e-14


def test_constant_images_closed_form_in_the_interior():
    """Constant images a, b: away from the border every variance is zero, so
    SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    x = np.full((30, 40), 0.3)
    y = np.full((30, 40), 0.7)
    m, _ = S.ssim_map(x, y)
    ref = (2 * 0.3 * 0.7 + S.C1) / (0.3 ** 2 + 0.7 ** 2 + S.C1)
    assert abs(m[10:20, 10:30] - ref).max() < 1e-12


def test_identical_images_give_one_and_zero_gradient():
    rng = np.random.default_rng(1)
    x = rng.random((3, 17, 23))
    val, (g,) = oracle.ssim([x], [x])
    assert abs(val - 1.0) < 1e-12
    assert np.abs(g).max() < 1e-12


def test_map_against_direct_window_sums():
    """The statistics written out pixel by pixel with explicit loops over the
    window (zero outside the image) give the same SSIM."""
    rng = np.random.default_rng(2)
    x, y = rng.random((9, 12)), rng.random((9, 12))
    w = S.window()
    H, W = x.shape
    ref = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            st = np.zeros(5)
            for di in range(-5, 6):
                for dj in range(-5, 6):
                    a, b = i + di, j + dj
                    if 0 <= a < H and 0 <= b < W:
                        ww = w[di + 5, dj + 5]
                        st += ww * np.array([x[a, b], y[a, b], x[a, b] ** 2, y[a, b] ** 2, x[a, b] * y[a, b]])
            mx, my = st[0], st[1]
            vx, vy, cxy = st[2] - mx * mx, st[3] - my * my, st[4] - mx * my
            ref[i, j] = (2 * mx * my + S.C1) * (2 * cxy + S.C2) / ((mx * mx + my * my + S.C1) * (vx + vy + S.C2))
    m, _ = S.ssim_map(x, y)
    assert np.abs(m - ref).max() < 1e-13


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    imgs = [rng.random((3, 13, 16)), rng.random((3, 9, 11))]
    tgts = [rng.random((3, 13, 16)), rng.random((3, 9, 11))]
    loss, grads = oracle.l1_dssim_loss(imgs, tgts)
    h = 1e-6
    for v in range(2):
        for idx in [(0, 0, 0), (1, 6, 7), (2, 8, 10), (0, 4, 1)]:
            if idx[1] >= imgs[v].shape[1] or idx[2] >= imgs[v].shape[2]:
                continue
            p = [a.copy() for a in imgs]
            m = [a.copy() for a in imgs]
            p[v][idx] += h
            m[v][idx] -= h
            fd = (oracle.l1_dssim_loss(p, tgts)[0] - oracle.l1_dssim_loss(m, tgts)[0]) / (2 * h)
            assert abs(fd - grads[v][idx]) < 1e-7 * max(abs(fd), 1e-3), (v, idx, fd, grads[v][idx])
