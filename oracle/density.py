"""Adaptive density control of 6D Gaussians, written out from its definition
(test infrastructure only).

Sec. 4.3: the 3D Gaussian splatting densification needs a scale and a rotation
per Gaussian, which the 6D form does not store.  They are taken from the
conditional covariance Sigma_cond (direction independent: a Schur complement)
by its SVD, Sigma_cond = U D U^T (for this symmetric positive definite matrix,
its eigendecomposition): R = U, S = sqrt(diag D), and the last column of R is
multiplied by sign(det R) so that R is a proper rotation.  The clone / split /
prune rules are those of 3DGS with the minimum opacity tau = 0.01 (Sec. 4.3,
Sec. 5.1).

Readings where the paper is silent (listed with the others in the design notes):
  * order: singular values descending (the SVD convention); signs: the first
    two axes with their largest component positive, the third their cross
    product (the paper's sign(det R) correction of the last column);
  * a Gaussian is densified when its mean screen-space gradient over the views
    it was visible in reaches ``grad_threshold`` (3DGS: 2e-4); it is cloned when
    max(S) <= ``percent_dense`` * ``extent`` (3DGS: 0.01 of the scene extent) and
    split otherwise; it is pruned when sigmoid(opacity logit) < ``min_opacity``;
  * clone: the Gaussian stays and an identical copy follows it;
  * split: the Gaussian is replaced by two whose spatial means are
    mu_p + R (S * z_k) for the standard normal draws z_0, z_1 (passed in), and
    whose spatial Cholesky block L_p is divided by 1.6 -- this divides
    Sigma_p by 1.6^2 and Sigma_pd by 1.6, so Sigma_cond is divided by 1.6^2
    (S by 1.6, R unchanged) while Sigma_d and the other parameters are kept;
  * outputs keep the parents' order, each parent's outputs consecutive; Adam
    moments are kept for kept and for the first (original) output of a clone,
    and are zero for clone copies and split children.
"""
from __future__ import annotations

import numpy as np

from . import NROWS, slice_gaussians

ROW_MU_P = 0
ROW_L = 6
ROW_OPA = 75
SPLIT_SCALE = 1.6
# storage index i(i+1)/2 + j of the spatial block L_p (rows and columns 0-2)
LP_DIAG = (0, 2, 5)
LP_OFF = (1, 3, 4)


def decompose(params):
    """R [N,3,3] (proper rotations) and S [N,3] (descending) with
    Sigma_cond = R diag(S^2) R^T."""
    p = np.asarray(params, np.float64)
    n = p.shape[1]
    dirs = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))  # any direction: Sigma_cond does not depend on it
    _, sig, _, _, _ = slice_gaussians(p, dirs, 0.35)
    w, U = np.linalg.eigh(sig)  # ascending
    w, U = w[:, ::-1], U[:, :, ::-1].copy()
    # the SVD fixes each axis only up to sign: the first two axes are taken with
    # their largest component positive, and the third as their cross product,
    # which is the paper's last-column sign(det R) correction
    for k in range(2):
        big = np.take_along_axis(U[:, :, k], np.argmax(np.abs(U[:, :, k]), axis=1)[:, None], axis=1)[:, 0]
        U[:, :, k] *= np.where(big < 0, -1.0, 1.0)[:, None]
    U[:, :, 2] = np.cross(U[:, :, 0], U[:, :, 1])
    return U, np.sqrt(np.clip(w, 0.0, None))


def decisions(params, stats, grad_threshold, percent_dense, extent, min_opacity):
    """Per Gaussian: 0 prune, 1 keep, 2 clone, 3 split; and the margins of the
    three threshold tests relative to their thresholds (for ambiguity checks)."""
    p = np.asarray(params, np.float64)
    st = np.asarray(stats, np.float64)
    _, S = decompose(p)
    alpha = 1.0 / (1.0 + np.exp(-p[ROW_OPA]))
    avg = np.where(st[1] > 0, st[0] / np.maximum(st[1], 1.0), 0.0)
    big = S.max(axis=1) > percent_dense * extent
    grow = avg >= grad_threshold
    d = np.where(alpha < min_opacity, 0, np.where(grow, np.where(big, 3, 2), 1))
    thr = percent_dense * extent
    size_margin = S.max(axis=1) / thr - 1.0 if thr > 0 else np.full(len(d), np.inf)
    margins = np.stack([alpha / min_opacity - 1.0, avg / grad_threshold - 1.0, size_margin])
    return d, margins


def densify(params, stats, noise, grad_threshold=2e-4, percent_dense=0.01, extent=1.0, min_opacity=0.01,
            m=None, v=None, lambda_raw=None):
    """Apply clone / split / prune.  ``stats`` is [2, N] (summed screen-space
    gradient norm, visible count), ``noise`` [2, 3, N] standard normal draws for
    the two children of a split.  Returns a dict with params [76, N'] and, when
    given, m, v ([76, N']) and lambda_raw ([N'])."""
    p = np.asarray(params, np.float64)
    n = p.shape[1]
    z = np.asarray(noise, np.float64).reshape(2, 3, n)
    R, S = decompose(p)
    d, _ = decisions(p, stats, grad_threshold, percent_dense, extent, min_opacity)
    cols, mcols, src = [], [], []
    for i in range(n):
        if d[i] == 0:
            continue
        if d[i] == 1:
            cols.append(p[:, i]); mcols.append(True); src.append(i)
        elif d[i] == 2:
            cols += [p[:, i], p[:, i]]; mcols += [True, False]; src += [i, i]
        else:
            for k in range(2):
                c = p[:, i].copy()
                c[ROW_MU_P:ROW_MU_P + 3] = p[ROW_MU_P:ROW_MU_P + 3, i] + R[i] @ (S[i] * z[k, :, i])
                for r in LP_DIAG:  # exp(raw) / 1.6
                    c[ROW_L + r] = p[ROW_L + r, i] - np.log(SPLIT_SCALE)
                for r in LP_OFF:  # (2 sigmoid(raw) - 1) / 1.6, back to raw
                    l = (2.0 / (1.0 + np.exp(-p[ROW_L + r, i])) - 1.0) / SPLIT_SCALE
                    c[ROW_L + r] = np.log((1.0 + l) / (1.0 - l))
                cols.append(c); mcols.append(False); src.append(i)
    out = {"params": np.stack(cols, 1) if cols else np.zeros((NROWS, 0)), "decisions": d}
    keep = np.array(mcols, bool)
    src = np.array(src, np.int64)
    for nm, a in (("m", m), ("v", v)):
        if a is not None:
            a = np.asarray(a, np.float64)
            o = np.zeros((NROWS, len(src)))
            o[:, keep] = a[:, src[keep]]
            out[nm] = o
    if lambda_raw is not None:
        out["lambda_raw"] = np.asarray(lambda_raw, np.float64)[src]
    return out
