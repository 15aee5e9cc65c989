"""Structural-similarity term of the training loss (test infrastructure only).

The paper trains with the 3D Gaussian splatting loss (Sec. 4.4, Sec. 5.1):
L = (1 - lambda) L1 + lambda (1 - SSIM) with lambda = 0.2.  SSIM (Wang et al.
2004) per channel and pixel from local statistics under an 11x11 Gaussian window
(sigma 1.5, weights summing to one), with C1 = 0.01^2 and C2 = 0.03^2 for a
data range of one; the window is zero-padded at the image border (as the 3DGS
code convolves) and SSIM is averaged over every channel and pixel of every view.

The gradient is written out by hand.  With the five local statistics
mu_x = w*x, mu_y = w*y, s_x = w*x^2 - mu_x^2, s_y = w*y^2 - mu_y^2,
s_xy = w*(xy) - mu_x mu_y and SSIM = f(mu_x, mu_y, s_x, s_y, s_xy):
  dSSIM/dx = w*(f_mu_x - 2 mu_x f_s_x - mu_y f_s_xy) + 2 x (w*f_s_x) + y (w*f_s_xy),
where w* is the correlation with the (symmetric) window restricted to the image.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WIN = 11
SIGMA = 1.5
LAMBDA_DSSIM = 0.2


def window():
    """The 11x11 Gaussian window (outer product of the normalised 1D one)."""
    t = np.arange(WIN) - WIN // 2
    g = np.exp(-t * t / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def _conv(a, w):
    return ndimage.correlate(a, w, mode="constant", cval=0.0)


def ssim_map(x, y):
    """SSIM per pixel of two single-channel images, and the partials of f
    needed by the gradient."""
    w = window()
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = _conv(x, w), _conv(y, w)
    sx = _conv(x * x, w) - mx * mx
    sy = _conv(y * y, w) - my * my
    sxy = _conv(x * y, w) - mx * my
    A1, A2 = 2 * mx * my + C1, 2 * sxy + C2
    B1, B2 = mx * mx + my * my + C1, sx + sy + C2
    S = A1 * A2 / (B1 * B2)
    # partials of S = A1 A2 / (B1 B2)
    f_mx = (2 * my * A2) / (B1 * B2) - S * (2 * mx) / B1
    f_sx = -S / B2
    f_sxy = 2 * A1 / (B1 * B2)
    return S, (mx, my, f_mx, f_sx, f_sxy)


def ssim(images, targets):
    """Mean SSIM over every channel and pixel of every view ([3, H, W] each),
    and dSSIM/dimage per view."""
    w = window()
    tot = sum(np.asarray(a).size for a in images)
    val = 0.0
    grads = []
    for img, tgt in zip(images, targets):
        img = np.asarray(img, np.float64)
        tgt = np.asarray(tgt, np.float64)
        g = np.zeros_like(img)
        for c in range(img.shape[0]):
            S, (mx, my, f_mx, f_sx, f_sxy) = ssim_map(img[c], tgt[c])
            val += S.sum()
            a = f_mx - 2 * mx * f_sx - my * f_sxy
            g[c] = (_conv(a, w) + 2 * img[c] * _conv(f_sx, w) + tgt[c] * _conv(f_sxy, w)) / tot
        grads.append(g)
    return val / tot, grads


def l1_dssim_loss(images, targets, lam=LAMBDA_DSSIM):
    """(1 - lam) L1 + lam (1 - SSIM) and its gradient per view."""
    from .train import l1_loss
    l1, g1 = l1_loss(images, targets)
    s, gs = ssim(images, targets)
    return (1 - lam) * l1 + lam * (1 - s), [(1 - lam) * a - lam * b for a, b in zip(g1, gs)]
