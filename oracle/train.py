"""Loss, optimiser and densification statistics as textbook definitions in
float64 (test infrastructure only).

The paper trains with the 3D Gaussian splatting losses and optimiser (Sec. 4.4,
Sec. 5.1: Adam, learning rate 1e-2 for the 6D covariance parameters and 1e-3 for
the direction mean, the 3DGS defaults elsewhere).  The training step measured
here uses the L1 term of that loss.
"""
from __future__ import annotations

import numpy as np

# Row ranges of the [76, N] parameter layout, one Adam learning rate per group.
GROUPS = [(0, 3), (3, 6), (6, 27), (27, 30), (30, 75), (75, 76)]


def l1_loss(images, targets):
    """mean |I - I*| over every view, channel and pixel, and dL/dI = sign(I - I*) / count."""
    imgs = [np.asarray(a, np.float64) for a in images]
    tgts = [np.asarray(b, np.float64) for b in targets]
    count = sum(a.size for a in imgs)
    loss = sum(np.abs(a - b).sum() for a, b in zip(imgs, tgts)) / count
    grads = [np.sign(a - b) / count for a, b in zip(imgs, tgts)]
    return loss, grads


def adam_step(params, grads, m, v, step: int, lrs, b1=0.9, b2=0.999, eps=1e-15):
    """One Adam step (Kingma and Ba, with bias correction) over the [76, N]
    layout; ``lrs`` holds one learning rate per row group.  Returns new
    (params, m, v)."""
    p = np.asarray(params, np.float64).copy()
    g = np.asarray(grads, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    for (r0, r1), lr in zip(GROUPS, lrs):
        p[r0:r1] -= lr * mh[r0:r1] / (np.sqrt(vh[r0:r1]) + eps)
    return p, m, v


def densify_stats(g2d_views, visible_views, cams):
    """Per Gaussian: sum over views of |(dL/du * W/2, dL/dv * H/2)| (the
    screen-space gradient in normalised device units) and the number of views
    in which it was visible."""
    n = g2d_views[0].shape[0]
    acc = np.zeros(n, np.float64)
    cnt = np.zeros(n, np.float64)
    for g2, vis, c in zip(g2d_views, visible_views, cams):
        nrm = np.hypot(g2[:, 0] * 0.5 * c.width, g2[:, 1] * 0.5 * c.height)
        acc += np.where(vis, nrm, 0.0)
        cnt += vis.astype(np.float64)
    return acc, cnt
