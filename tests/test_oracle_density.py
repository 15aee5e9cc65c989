"""Pins of the oracle's adaptive density control (CPU only): the SVD-based
rotation and scale of Sec. 4.3 against closed forms and sampling, and the
clone / split / prune rules on a hand-made set."""
import math

import numpy as np

import oracle
import synth

ROW_L, ROW_OPA = 6, 75


def _scene(n, seed):
    spec = synth.SceneSpec(n=n, seed=seed, l_cross_std=0.4)
    return synth.make_scene(spec).astype(np.float64)


def test_decompose_reconstructs_sigma_cond_with_proper_rotations():
    p = _scene(500, 3)
    R, S = oracle.decompose(p)
    dirs = np.tile([0.0, 0.0, 1.0], (p.shape[1], 1))
    _, sig, _, _, _ = oracle.slice_gaussians(p, dirs, 0.35)
    rec = np.einsum("nij,nj,nkj->nik", R, S ** 2, R)
    assert np.abs(rec - sig).max() <= 1e-12 * np.abs(sig).max()
    assert np.abs(np.einsum("nji,njk->nik", R, R) - np.eye(3)).max() < 1e-12
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-12)
    assert np.all(S[:, 0] >= S[:, 1]) and np.all(S[:, 1] >= S[:, 2]) and np.all(S >= 0)


def test_decompose_of_axis_aligned_spatial_gaussian():
    """No cross terms and a diagonal L_p: Sigma_cond = diag(exp(2 raw)), so S is
    exp(raw) sorted and R the matching (proper) permutation."""
    p = np.zeros((76, 1))
    p[ROW_L + 0, 0], p[ROW_L + 2, 0], p[ROW_L + 5, 0] = -2.0, -1.0, -3.0   # L_00, L_11, L_22 raw
    p[ROW_L + 9, 0] = p[ROW_L + 14, 0] = p[ROW_L + 20, 0] = -1.0          # direction diagonal
    R, S = oracle.decompose(p)
    assert np.allclose(S[0], np.exp([-1.0, -2.0, -3.0]), rtol=1e-12)
    assert np.allclose(np.abs(R[0]), [[0, 1, 0], [1, 0, 0], [0, 0, 1]], atol=1e-12)
    assert abs(np.linalg.det(R[0]) - 1.0) < 1e-12


def test_split_children_sample_sigma_cond_and_shrink_it_by_1_6():
    """One Gaussian split with many draws: the children's means scatter with the
    parent's Sigma_cond (sampling check), and each child's Sigma_cond is the
    parent's over 1.6^2 with the same axes; its direction block is untouched."""
    p1 = _scene(1, 11)
    m = 20000
    p = np.repeat(p1, m, axis=1)
    stats = np.stack([np.ones(m), np.ones(m)])
    z = np.random.default_rng(5).normal(size=(2, 3, m))
    out = oracle.densify(p, stats, z, grad_threshold=0.5, percent_dense=0.0, extent=1.0)
    assert np.all(out["decisions"] == 3) and out["params"].shape[1] == 2 * m
    kids = out["params"]
    R, S = oracle.decompose(p1)
    sig = R[0] @ np.diag(S[0] ** 2) @ R[0].T
    cov = np.cov(kids[0:3] - p1[0:3], bias=False)
    assert np.abs(cov - sig).max() < 0.05 * np.abs(sig).max()
    Rk, Sk = oracle.decompose(kids[:, :1])
    assert np.allclose(Sk[0], S[0] / 1.6, rtol=1e-10)
    assert np.allclose(np.abs(Rk[0].T @ R[0]), np.eye(3), atol=1e-8)
    d = np.array([[0.3, -0.5, 0.81]]) / np.linalg.norm([0.3, -0.5, 0.81])
    _, _, D0, _, _ = oracle.slice_gaussians(p1, d, 0.35)
    _, _, D1, _, _ = oracle.slice_gaussians(kids[:, :1], d, 0.35)
    assert abs(D0[0] - D1[0]) < 1e-12 * max(abs(D0[0]), 1.0)


def test_clone_split_prune_keep_by_hand():
    p = _scene(5, 17)
    p[ROW_OPA] = [2.0, 2.0, 2.0, 2.0, math.log(0.005 / 0.995)]  # last: opacity 0.005 < 0.01
    _, S = oracle.decompose(p)
    extent = 1.0
    pd = float(np.median(S.max(axis=1)[:4]))  # thresholds between the four maxima
    smax = S.max(axis=1)
    stats = np.array([[3e-4, 3e-4, 1e-4, 0.0, 9e-4], [1.0, 1.0, 1.0, 0.0, 1.0]])
    z = np.random.default_rng(2).normal(size=(2, 3, 5))
    m = np.random.default_rng(3).normal(size=(76, 5))
    lam = np.arange(5.0)
    out = oracle.densify(p, stats, z, grad_threshold=2e-4, percent_dense=pd, extent=extent, m=m, v=m ** 2,
                         lambda_raw=lam)
    expect = []
    for i in range(5):
        if i == 4:
            expect.append(0)
        elif stats[0, i] >= 2e-4:
            expect.append(3 if smax[i] > pd * extent else 2)
        else:
            expect.append(1)
    assert list(out["decisions"]) == expect
    sizes = {0: 0, 1: 1, 2: 2, 3: 2}
    assert out["params"].shape[1] == sum(sizes[d] for d in expect)
    col = 0
    for i, d in enumerate(expect):
        if d == 1:
            assert np.array_equal(out["params"][:, col], p[:, i]) and np.array_equal(out["m"][:, col], m[:, i])
        if d == 2:
            assert np.array_equal(out["params"][:, col], p[:, i]) and np.array_equal(out["params"][:, col + 1], p[:, i])
            assert np.array_equal(out["m"][:, col], m[:, i]) and not out["m"][:, col + 1].any()
        if d == 3:
            assert not out["m"][:, col].any() and not out["v"][:, col + 1].any()
            assert np.array_equal(out["params"][27:, col], p[27:, i])  # SH and opacity copied
        assert all(out["lambda_raw"][col + k] == lam[i] for k in range(sizes[d]))
        col += sizes[d]
