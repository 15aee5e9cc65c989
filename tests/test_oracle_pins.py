"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these retypes the oracle's own formulas: each compares it with an
independent route (a library routine, a different closed form, an analytic
special case, finite differences or brute force).
"""
import math

import numpy as np
import pytest
import scipy.special
import torch

import oracle
import synth

LAM = 0.35


def blank(n):
    """Raw parameters with every Cholesky off-diagonal at raw 0 (activated 0)."""
    return np.zeros((76, n), np.float64)


def tanh_half(x):
    return np.tanh(0.5 * x)  # equals 2 sigmoid(x) - 1


def activated_L(p, i):
    L = np.zeros((6, 6))
    for r in range(6):
        for c in range(r + 1):
            raw = p[6 + r * (r + 1) // 2 + c, i]
            L[r, c] = math.exp(raw) if r == c else tanh_half(raw)
    return L


def random_gaussians(n, seed, cross=0.4):
    rng = np.random.default_rng(seed)
    p = np.zeros((76, n))
    p[0:3] = rng.uniform(-0.5, 0.5, (3, n))
    d = rng.normal(size=(3, n))
    p[3:6] = d / np.linalg.norm(d, axis=0)
    for k in range(21):
        if k in synth.DIAG_SPATIAL:
            p[6 + k] = rng.normal(-2.0, 0.3, n)
        elif k in synth.DIAG_DIRECTION:
            p[6 + k] = rng.normal(-0.8, 0.2, n)
        elif k in synth.CROSS_BLOCK:
            p[6 + k] = rng.normal(0.0, cross, n)
        else:
            p[6 + k] = rng.normal(0.0, 0.3, n)
    p[27:75] = rng.normal(0, 0.3, (48, n))
    p[75] = rng.normal(0.5, 1.0, n)
    return p


def unit_dirs(n, seed):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


# ----------------------------------------------------------------- SH basis
def test_sh_orthonormal_by_quadrature():
    """Real SH of degree <= 3 are orthonormal on the sphere (Sec. 4.2 colour basis)."""
    x, w = np.polynomial.legendre.leggauss(16)
    nphi = 32
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    Y = oracle.sh_basis(dirs)
    gram = Y.T @ (wts[:, None] * Y)
    assert np.abs(gram - np.eye(16)).max() < 1e-12


def test_sh_matches_scipy_up_to_sign():
    """Each basis function equals scipy's real SH (l, m) up to one global sign
    per function; the order is k = l^2 + l + m."""
    dirs = unit_dirs(200, 7)
    theta = np.arccos(dirs[:, 2])
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    Y = oracle.sh_basis(dirs)
    for l in range(4):
        for m in range(-l, l + 1):
            c = scipy.special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * c.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * c.imag
            else:
                ref = c.real
            k = l * l + l + m
            s = np.sign(np.dot(Y[:, k], ref))
            assert s != 0
            assert np.abs(Y[:, k] - s * ref).max() < 1e-12, (l, m)


# ---------------------------------------------------------------- the slice
def test_slice_matches_precision_form_and_woodbury():
    """eq:mu / eq:sigma against the precision-matrix form of a Gaussian
    conditional and against the Woodbury form L_p (I + M^T M)^-1 L_p^T."""
    n = 64
    p = random_gaussians(n, 1)
    dirs = unit_dirs(n, 2)
    for lam in (0.0, LAM, 1.0):
        mu_c, sig_c, D, f, ac = oracle.slice_gaussians(p, dirs, lam)
        for i in range(n):
            L = activated_L(p, i)
            S = L @ L.T
            Lam = np.linalg.inv(S)
            x = dirs[i] - p[3:6, i]
            sc_ref = np.linalg.inv(Lam[:3, :3])
            mu_ref = p[0:3, i] - sc_ref @ Lam[:3, 3:] @ x
            M = np.linalg.solve(L[3:, 3:], L[3:, :3])
            wood = L[:3, :3] @ np.linalg.inv(np.eye(3) + M.T @ M) @ L[:3, :3].T
            D_ref = x @ np.linalg.solve(S[3:, 3:], x)
            assert np.allclose(sig_c[i], sc_ref, rtol=1e-10, atol=1e-14)
            assert np.allclose(sig_c[i], wood, rtol=1e-10, atol=1e-14)
            assert np.allclose(mu_c[i], mu_ref, rtol=1e-10, atol=1e-13)
            assert abs(D[i] - D_ref) <= 1e-10 * max(1.0, D_ref)
            alpha = 1.0 / (1.0 + math.exp(-p[75, i]))
            assert abs(f[i] - math.exp(-lam * D_ref)) < 1e-12
            assert abs(ac[i] - alpha * math.exp(-lam * D_ref)) < 1e-12


def test_conditional_opacity_curve_special_cases():
    """Sec. 5 (fig. on f_cond): lambda = 0 gives f = 1, lambda = 1 the N-DG form
    exp(-D) of eq:pdf; f decreases with D."""
    n = 32
    p = random_gaussians(n, 3)
    dirs = unit_dirs(n, 4)
    _, _, D0, f0, _ = oracle.slice_gaussians(p, dirs, 0.0)
    assert np.all(f0 == 1.0)
    _, _, D1, f1, _ = oracle.slice_gaussians(p, dirs, 1.0)
    assert np.allclose(f1, np.exp(-D1), rtol=1e-14)
    _, _, D2, f2, _ = oracle.slice_gaussians(p, dirs, LAM)
    order = np.argsort(D2)
    assert np.all(np.diff(f2[order]) <= 0)


def test_sigma_cond_independent_of_direction():
    """Sec. 4.1: the conditional covariance does not depend on d."""
    p = random_gaussians(16, 5)
    _, s1, _, _, _ = oracle.slice_gaussians(p, unit_dirs(16, 6), LAM)
    _, s2, _, _, _ = oracle.slice_gaussians(p, unit_dirs(16, 7), LAM)
    assert np.array_equal(s1, s2)


def test_conditional_mean_is_regression_by_sampling():
    """mu_cond is E[X_p | X_d = d]: a least-squares fit of X_p on X_d over
    samples of the 6D Gaussian recovers the same linear map (tolerance set by
    the Monte-Carlo error)."""
    p = random_gaussians(1, 11, cross=0.8)
    L = activated_L(p, 0)
    rng = np.random.default_rng(0)
    X = rng.normal(size=(400_000, 6)) @ L.T
    Xp, Xd = X[:, :3], X[:, 3:]
    B, *_ = np.linalg.lstsq(np.c_[Xd, np.ones(len(X))], Xp, rcond=None)
    d = unit_dirs(1, 12)
    mu_c, _, _, _, _ = oracle.slice_gaussians(p, d, LAM)
    # the fitted map is for zero-mean variables; shift by the means
    x = d[0] - p[3:6, 0]
    pred = p[0:3, 0] + B[:3].T @ x
    resid = Xp - np.c_[Xd, np.ones(len(X))] @ B
    sc_mc = resid.T @ resid / len(X)
    _, sc, _, _, _ = oracle.slice_gaussians(p, d, LAM)
    scale = np.abs(sc[0]).max()
    assert np.allclose(mu_c[0], pred, atol=0.02 * math.sqrt(scale) * (1 + np.linalg.norm(x)))
    assert np.allclose(sc[0], sc_mc, atol=0.03 * scale)


# ------------------------------------------------------ single / two Gaussians
def axis_scene(depths, sigmas, logits, dc, cam, mu_d_equal_view=True):
    """Gaussians on the optical axis: L_p = s I, L_dp = 0, degree-0 SH only."""
    n = len(depths)
    p = blank(n)
    C = cam.center
    fwd = cam.R[2]
    for i in range(n):
        p[0:3, i] = C + depths[i] * fwd
        p[3:6, i] = fwd if mu_d_equal_view else -fwd
        for k in synth.DIAG_SPATIAL:
            p[6 + k, i] = math.log(sigmas[i])
        for k in synth.DIAG_DIRECTION:
            p[6 + k, i] = math.log(0.5)
        p[75, i] = logits[i]
        for c in range(3):
            p[27 + c, i] = dc[i][c]
    return p


def exact_camera(W, H, center=(0.1, -3.0, 0.2), f=None):
    """Camera looking along +y with an exactly orthonormal rotation."""
    R = np.array([[1.0, 0, 0], [0, 0, -1.0], [0, 1.0, 0]])
    c = np.asarray(center, np.float64)
    f = f if f is not None else 0.9 * W
    return synth.Camera(R, -R @ c, f, f, W / 2.0, H / 2.0, W, H)


def analytic_alpha(cam, depth, sigma, alpha, settings):
    """a at every pixel for an on-axis isotropic Gaussian (slice is the identity,
    Sigma_2D = ((f s / z)^2 + 0.3) I)."""
    H, W = cam.height, cam.width
    jj, ii = np.mgrid[0:H, 0:W]
    r2 = (ii + 0.5 - cam.cx) ** 2 + (jj + 0.5 - cam.cy) ** 2
    s2 = (cam.fx * sigma / depth) ** 2 + settings.dilation
    a = np.minimum(settings.alpha_max, alpha * np.exp(-0.5 * r2 / s2))
    return np.where(a >= settings.alpha_min, a, 0.0)


def test_single_gaussian_analytic_image():
    cam = exact_camera(64, 48)
    st = oracle.Settings(bg=(0.2, 0.3, 0.4))
    depth, sigma, logit = 3.0, 0.05, 0.7
    dc = (0.5, -1.0, 2.0)
    p = axis_scene([depth], [sigma], [logit], [dc], cam)
    img, T, nc, amb = oracle.render(p, cam, st)
    a = analytic_alpha(cam, depth, sigma, 1 / (1 + math.exp(-logit)), st)
    Y0 = 0.5 / math.sqrt(math.pi)
    for c in range(3):
        col = 1 / (1 + math.exp(-dc[c] * Y0))
        ref = col * a + st.bg[c] * (1 - a)
        assert np.abs(img[c] - ref).max() < 1e-12
    assert np.abs(T - (1 - a)).max() < 1e-12
    assert np.array_equal(nc, (a > 0).astype(np.int64))
    # the record: projection to the principal point, dilated isotropic footprint
    r = oracle.preprocess(p, cam, st)
    assert abs(r["u"][0] - cam.cx) < 1e-9 and abs(r["v"][0] - cam.cy) < 1e-9
    s2 = (cam.fx * sigma / depth) ** 2 + 0.3
    assert np.allclose(r["cov2d"][0], [s2, 0, s2], atol=1e-9)


def test_two_gaussians_composite_in_depth_order():
    """C = c1 a1 + c2 a2 (1 - a1) + bg (1 - a1)(1 - a2), front one first, even
    when it has the higher index; equal depths go by index."""
    cam = exact_camera(40, 40, center=(0.0, -2.0, 0.5))
    st = oracle.Settings(bg=(0.1, 0.1, 0.1))
    Y0 = 0.5 / math.sqrt(math.pi)
    for depths, front in (([3.5, 2.5], 1), ([2.5, 3.5], 0), ([3.0, 3.0], 0)):
        sig = [0.06, 0.04]
        logits = [1.5, 0.2]
        dcs = [(2.0, -2.0, 0.0), (-1.0, 3.0, 1.0)]
        p = axis_scene(depths, sig, logits, dcs, cam)
        img, T, nc, _ = oracle.render(p, cam, st)
        a = [analytic_alpha(cam, depths[i], sig[i], 1 / (1 + math.exp(-logits[i])), st) for i in range(2)]
        col = [[1 / (1 + math.exp(-dcs[i][c] * Y0)) for c in range(3)] for i in range(2)]
        f, b = front, 1 - front
        for c in range(3):
            ref = col[f][c] * a[f] + col[b][c] * a[b] * (1 - a[f]) + st.bg[c] * (1 - a[f]) * (1 - a[b])
            assert np.abs(img[c] - ref).max() < 1e-12


def test_early_termination_before_t_min():
    """Stacked opaque Gaussians: the walk stops before T would fall below 1e-4."""
    cam = exact_camera(16, 16)
    st = oracle.Settings()
    n = 6
    depths = [2.0 + 0.1 * i for i in range(n)]
    p = axis_scene(depths, [0.2] * n, [8.0] * n, [(0.0, 0.0, 0.0)] * n, cam)
    _, T, nc, _ = oracle.render(p, cam, st)
    alpha = 1 / (1 + math.exp(-8.0))
    a = [analytic_alpha(cam, d, 0.2, alpha, st) for d in depths]
    Tref = np.ones_like(a[0])
    nref = np.zeros_like(a[0], dtype=np.int64)
    stopped = np.zeros_like(a[0], dtype=bool)
    for k in range(n):
        Tn = Tref * (1 - a[k])
        take = ~stopped & (a[k] > 0) & (Tn >= st.t_min)
        stopped |= ~stopped & (a[k] > 0) & (Tn < st.t_min)
        Tref = np.where(take, Tn, Tref)
        nref += take
    assert np.abs(T - Tref).max() < 1e-12
    assert np.array_equal(nc, nref)
    assert stopped.any()  # termination actually happened somewhere


# --------------------------------------------------- projection / 3DGS limit
def pinhole(cam, X):
    p = cam.R @ X + cam.t
    return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])


def test_projection_matches_finite_difference_jacobian():
    """With L_dp = 0 the slice leaves mu_p and Sigma_p unchanged (3DGS limit,
    Sec. 4.4); u, v is the pinhole image of the mean and the 2D covariance is
    J Sigma J^T + 0.3 I with J the Jacobian of the pinhole map, here taken by
    central differences."""
    cam = synth.default_camera(200, 150)
    p = random_gaussians(20, 21, cross=0.0)
    for k in synth.CROSS_BLOCK:
        p[6 + k] = 0.0
    r = oracle.preprocess(p, cam)
    for i in range(20):
        X = p[0:3, i]
        uv = pinhole(cam, X)
        assert np.allclose([r["u"][i], r["v"][i]], uv, atol=1e-9)
        J = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3); e[k] = 1e-6
            J[:, k] = (pinhole(cam, X + e) - pinhole(cam, X - e)) / 2e-6
        L = activated_L(p, i)
        S = (L @ L.T)[:3, :3]
        assert np.allclose(r["sigma_cond"][i], S[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]], atol=1e-14)
        c2 = J @ S @ J.T + 0.3 * np.eye(2)
        assert np.allclose(r["cov2d"][i], [c2[0, 0], c2[0, 1], c2[1, 1]], rtol=1e-6)
        Q = np.linalg.inv(c2)
        assert np.allclose(r["conic"][i], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-6)


def test_large_direction_covariance_removes_view_dependence():
    """With Sigma_d = (1e3)^2 I the slice tends to the plain 3D Gaussian:
    the image no longer depends on mu_d or on the cross block, and equals the
    render with L_dp = 0 and lambda = 0 to O(lambda/s^2)."""
    w = synth.workload("c0", n_override=200)
    base = synth.make_scene(w.scene).astype(np.float64)
    cam = synth.default_camera(96, 96)
    big = base.copy()
    for k in synth.DIAG_DIRECTION:
        big[6 + k] = math.log(1e3)
    for k in synth.OFFDIAG_DIRECTION:
        big[6 + k] = 0.0
    ref_p = big.copy()
    for k in synth.CROSS_BLOCK:
        ref_p[6 + k] = 0.0
    img_big, *_ = oracle.render(big, cam)
    img_ref, *_ = oracle.render(ref_p, cam, oracle.Settings(lambda_opa=0.0))
    assert np.abs(img_big - img_ref).max() < 1e-4
    flipped = big.copy()
    flipped[3:6] *= -1
    img_flip, *_ = oracle.render(flipped, cam)
    assert np.abs(img_big - img_flip).max() < 1e-5


def test_extent_box_contains_every_contributing_pixel():
    """The opacity-aware box (q <= 2 ln(255 alpha_cond)) holds every pixel
    where a >= 1/255, checked by brute force over the whole frame."""
    w = synth.workload("c0")
    p = synth.make_scene(w.scene)
    cam = w.cameras[0]
    r = oracle.preprocess(p, cam)
    H, W = cam.height, cam.width
    jj, ii = np.mgrid[0:H, 0:W]
    px, py = ii + 0.5, jj + 0.5
    checked = 0
    for i in np.nonzero(r["alive"])[0]:
        dx, dy = px - r["u"][i], py - r["v"][i]
        qa, qb, qc = r["conic"][i]
        a = np.minimum(0.99, r["alpha_cond"][i] * np.exp(-0.5 * (qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy)))
        hit = a >= 1 / 255
        inside = (np.abs(dx) <= r["ex"][i]) & (np.abs(dy) <= r["ey"][i])
        assert not np.any(hit & ~inside)
        checked += hit.sum()
    assert checked > 1000


# ------------------------------------------------------------- backward pins
def record_vector(r):
    """(u, v, Qxx, Qxy, Qyy, alpha_cond, r, g, b) per Gaussian."""
    return np.c_[r["u"], r["v"], r["conic"], r["alpha_cond"], r["rgb"]]


def test_record_vjp_matches_finite_differences():
    """Chain rule through projection (both clamped and unclamped Jacobian
    guard), SH colour, slice, Cholesky and activations, against central
    differences of the oracle's own forward record."""
    cam = synth.default_camera(120, 90)
    n = 8
    p = random_gaussians(n, 31)
    # push two Gaussians outside the 1.3 guard in x and y (clamped Jacobian)
    right = cam.R[0]
    down = cam.R[1]
    p[0:3, 0] += 2.2 * right
    p[0:3, 1] += 2.0 * down
    st = oracle.Settings(lambda_opa=LAM)
    r0 = oracle.preprocess(p, cam, st)
    assert r0["alive"].all()
    wts = np.random.default_rng(5).normal(size=(n, 9))

    def loss(pp):
        rv = record_vector(oracle.preprocess(pp, cam, st))
        full = wts.copy()
        full[:, 3] *= 2.0  # dL/dQxy counts the two symmetric entries
        return float((rv * full).sum())

    g = oracle.record_vjp(p, cam, wts, st)
    fd = np.zeros_like(g)
    for row in range(76):
        for i in range(n):
            h = 1e-6 * max(1.0, abs(p[row, i]))
            pp = p.copy(); pp[row, i] += h
            pm = p.copy(); pm[row, i] -= h
            fd[row, i] = (loss(pp) - loss(pm)) / (2 * h)
    err = np.abs(g - fd)
    assert err.max() <= 1e-6 * max(1.0, np.abs(fd).max()), err.max()
    assert np.abs(g).max() > 1e-3


def tiny_scene(n, seed, W=28, H=24):
    rng = np.random.default_rng(seed)
    p = random_gaussians(n, seed)
    p[0:3] = rng.uniform(-0.25, 0.25, (3, n))
    for k in synth.DIAG_SPATIAL:
        p[6 + k] = rng.normal(-2.3, 0.2, n)
    cam = synth.look_at_camera((0.4, -2.5, 0.6), W, H, fov_x_deg=40.0)
    return p, cam


def test_backward_matches_finite_differences_on_tiny_scene():
    """Analytic backward of the whole render (reverse compositing and the
    per-Gaussian chain) against FP64 central differences; estimates where the
    h and h/2 differences disagree (a threshold crossed) are discarded."""
    n = 6
    p, cam = tiny_scene(n, 41)
    st = oracle.Settings(bg=(0.3, 0.2, 0.1))
    w = np.random.default_rng(9).normal(size=(3, cam.height, cam.width))

    def loss(pp):
        img, *_ = oracle.render(pp, cam, st, nthreads=1)
        return float((img * w).sum())

    g, _ = oracle.backward(p, cam, w, st, nthreads=1)
    fd = np.full_like(g, np.nan)
    discarded = 0
    for row in range(76):
        for i in range(n):
            h = 1e-6 * max(1.0, abs(p[row, i]))
            est = []
            for hh in (h, h / 2):
                pp = p.copy(); pp[row, i] += hh
                pm = p.copy(); pm[row, i] -= hh
                est.append((loss(pp) - loss(pm)) / (2 * hh))
            if abs(est[0] - est[1]) > 0.1 * max(abs(est[1]), 1e-3):
                discarded += 1
                continue
            fd[row, i] = est[1]
    ok = ~np.isnan(fd)
    assert ok.sum() >= 0.9 * ok.size, discarded
    scale = np.abs(fd[ok]).max()
    assert scale > 1e-2
    assert np.abs(g[ok] - fd[ok]).max() <= 1e-5 * scale
    for r0, r1 in ((0, 3), (3, 6), (6, 27), (27, 75), (75, 76)):
        sel = ok[r0:r1]
        a, b = g[r0:r1][sel], fd[r0:r1][sel]
        if np.linalg.norm(b) > 1e-6:
            assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)


def test_per_gaussian_lambda_constant_equals_scalar_setting():
    """A per-Gaussian lambda array holding the scalar value everywhere renders
    and differentiates exactly like the scalar setting (the learnable-lambda
    path changes where lambda comes from, nothing else)."""
    p, cam = tiny_scene(6, 47)
    st = oracle.Settings(bg=(0.3, 0.2, 0.1), lambda_opa=0.35)
    raw = np.full(p.shape[1], math.log(0.35 / 0.65))
    w = np.random.default_rng(5).normal(size=(3, cam.height, cam.width))
    img_s, T_s, *_ = oracle.render(p, cam, st, nthreads=1)
    img_a, T_a, *_ = oracle.render(p, cam, st, nthreads=1, lambda_raw=raw)
    assert np.abs(img_s - img_a).max() < 1e-13 and np.abs(T_s - T_a).max() < 1e-13
    g_s, _ = oracle.backward(p, cam, w, st, nthreads=1)
    g_a, _, g_lam = oracle.backward(p, cam, w, st, nthreads=1, lambda_raw=raw)
    assert np.abs(g_s - g_a).max() <= 1e-12 * max(np.abs(g_s).max(), 1.0)
    assert np.abs(g_lam).max() > 0


def test_lambda_gradient_matches_finite_differences():
    """dL/dlambda_raw of the whole render against FP64 central differences,
    with a different lambda per Gaussian; lambda -> 0 (raw -> -inf) must
    remove the view dependence of the opacity, so its gradient vanishes."""
    n = 6
    p, cam = tiny_scene(n, 53)
    st = oracle.Settings(bg=(0.1, 0.3, 0.2))
    raw = np.random.default_rng(6).normal(0.0, 1.0, n)
    w = np.random.default_rng(7).normal(size=(3, cam.height, cam.width))

    def loss(r):
        img, *_ = oracle.render(p, cam, st, nthreads=1, lambda_raw=r)
        return float((img * w).sum())

    _, _, g = oracle.backward(p, cam, w, st, nthreads=1, lambda_raw=raw)
    fd = []
    for i in range(n):
        h = 1e-6
        est = []
        for hh in (h, h / 2):
            rp = raw.copy(); rp[i] += hh
            rm = raw.copy(); rm[i] -= hh
            est.append((loss(rp) - loss(rm)) / (2 * hh))
        assert abs(est[0] - est[1]) <= 0.1 * max(abs(est[1]), 1e-6)
        fd.append(est[1])
    fd = np.array(fd)
    assert np.abs(fd).max() > 1e-3
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max()
    _, _, g0 = oracle.backward(p, cam, w, st, nthreads=1, lambda_raw=np.full(n, -60.0))
    assert np.abs(g0).max() < 1e-20


def test_backward_pixel_subset_is_restriction_of_full_frame():
    """The gradient of a loss on a pixel subset equals the full-frame gradient
    with the upstream gradient zero elsewhere."""
    p, cam = tiny_scene(5, 43)
    pix = synth.pixel_subset(cam.width, cam.height, 100, seed=4)
    w = np.random.default_rng(2).normal(size=(len(pix), 3))
    full = np.zeros((3, cam.height * cam.width))
    full[:, pix] = w.T
    g_sub, _ = oracle.backward(p, cam, w, pixels=pix)
    g_full, _ = oracle.backward(p, cam, full.reshape(3, cam.height, cam.width))
    assert np.allclose(g_sub, g_full, rtol=1e-12, atol=1e-14)


# ------------------------------------------------------- integer stage pins
def test_binning_against_brute_force_per_tile():
    """Tile lists: for every tile, the entries whose rectangle covers it, in
    (float32 depth bits, entry id) order, found by a direct scan."""
    rng = np.random.default_rng(17)
    cams = [synth.default_camera(70, 50), synth.default_camera(33, 65)]
    n = 300
    E = n * len(cams)
    u = rng.uniform(-20, 90, E).astype(np.float32)
    v = rng.uniform(-20, 90, E).astype(np.float32)
    ex = rng.exponential(6, E).astype(np.float32)
    ey = rng.exponential(6, E).astype(np.float32)
    depth = rng.choice(np.float32([1.0, 1.5, 2.25, 3.0]), E).astype(np.float32)  # many ties
    alive = rng.random(E) < 0.8
    for tw, th in ((16, 16), (32, 8), (8, 8)):
        out = oracle.bin_records(u, v, ex, ey, depth, alive, n, cams, tw, th)
        grid, total = oracle.tile_grid(cams, tw, th)
        assert out["ranges"].shape == (total, 2)
        for vi, (ntx, nty, base) in enumerate(grid):
            for ty in range(nty):
                for tx in range(ntx):
                    lst = []
                    for e in range(vi * n, (vi + 1) * n):
                        if not alive[e]:
                            continue
                        x0 = min(max(math.floor(float(np.float32(u[e] - ex[e])) / tw), 0), ntx)
                        x1 = min(max(math.floor(float(np.float32(u[e] + ex[e])) / tw) + 1, 0), ntx)
                        y0 = min(max(math.floor(float(np.float32(v[e] - ey[e])) / th), 0), nty)
                        y1 = min(max(math.floor(float(np.float32(v[e] + ey[e])) / th) + 1, 0), nty)
                        if x0 <= tx < x1 and y0 <= ty < y1:
                            lst.append((float(depth[e]), e))
                    lst.sort()
                    s, t = out["ranges"][base + ty * ntx + tx]
                    assert [e for _, e in lst] == list(out["values"][s:t])
                    keys = out["keys"][s:t]
                    assert all(int(k) >> 32 == base + ty * ntx + tx for k in keys)


# ------------------------------------------------------- loss / optimiser pins
def test_l1_matches_torch():
    rng = np.random.default_rng(0)
    imgs = [rng.random((3, 5, 7)), rng.random((3, 4, 4))]
    tgts = [rng.random((3, 5, 7)), imgs[1].copy()]
    tgts[1][0, 0, 0] += 0.5
    loss, grads = oracle.l1_loss(imgs, tgts)
    ti = [torch.tensor(a, requires_grad=True) for a in imgs]
    flat = torch.cat([a.reshape(-1) for a in ti])
    ref = torch.nn.functional.l1_loss(flat, torch.cat([torch.tensor(b).reshape(-1) for b in tgts]))
    ref.backward()
    assert abs(loss - ref.item()) < 1e-15
    for g, t in zip(grads, ti):
        assert np.allclose(g, t.grad.numpy(), atol=1e-18)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(1)
    n = 50
    p = rng.normal(size=(76, n))
    lrs = [1.6e-4, 1e-3, 1e-2, 2.5e-3, 1.25e-4, 5e-2]
    from oracle.train import GROUPS
    tp = [torch.tensor(p[a:b].copy(), requires_grad=True) for a, b in GROUPS]
    opt = torch.optim.Adam([{"params": [t], "lr": lr} for t, lr in zip(tp, lrs)], betas=(0.9, 0.999), eps=1e-15)
    m = np.zeros_like(p); v = np.zeros_like(p)
    cur = p.copy()
    for step in range(1, 6):
        g = rng.normal(size=p.shape)
        cur, m, v = oracle.adam_step(cur, g, m, v, step, lrs)
        for t, (a, b) in zip(tp, GROUPS):
            t.grad = torch.tensor(g[a:b].copy())
        opt.step()
    ref = np.concatenate([t.detach().numpy() for t in tp])
    assert np.allclose(cur, ref, rtol=1e-12, atol=1e-15)


def test_densify_stats_by_hand():
    cams = [synth.default_camera(100, 50), synth.default_camera(20, 40)]
    g1 = np.zeros((2, 9)); g1[0, :2] = [0.3, 0.4]; g1[1, :2] = [1.0, 0.0]
    g2 = np.zeros((2, 9)); g2[0, :2] = [0.0, 0.5]; g2[1, :2] = [9.0, 9.0]
    acc, cnt = oracle.densify_stats([g1, g2], [np.array([True, True]), np.array([True, False])], cams)
    assert np.allclose(acc, [math.hypot(0.3 * 50, 0.4 * 25) + 0.5 * 20, 50.0])
    assert np.allclose(cnt, [2, 1])


# ------------------------------------------------- No-SH colour (Sec. 5 ablation)
Y00 = 0.5 / math.sqrt(math.pi)  # the degree-0 real spherical harmonic, 1 / (2 sqrt(pi))


def test_rgb_color_equals_dc_only_sh():
    """The per-Gaussian RGB colour rgb = sigmoid(c) renders exactly like the SH
    colour with only degree-0 coefficients beta0 = c / Y00 (the degree-0
    harmonic is the constant 1 / (2 sqrt(pi))), which the quadrature and scipy
    pins fix; the RGB path itself evaluates no harmonic at all."""
    p, cam = tiny_scene(6, 61)
    c = np.random.default_rng(8).normal(0.0, 1.0, (3, p.shape[1]))
    p_rgb = p.copy()
    p_rgb[27:30] = c
    p_rgb[30:75] = np.random.default_rng(9).normal(0.0, 5.0, (45, p.shape[1]))  # unused in RGB mode
    p_sh = p.copy()
    p_sh[27:30] = c / Y00
    p_sh[30:75] = 0.0
    img_rgb, T_rgb, *_ = oracle.render(p_rgb, cam, oracle.Settings(rgb_color=True), nthreads=1)
    img_sh, T_sh, *_ = oracle.render(p_sh, cam, oracle.Settings(), nthreads=1)
    assert np.abs(img_rgb - img_sh).max() < 1e-12 and np.abs(T_rgb - T_sh).max() < 1e-13
    assert img_rgb.max() > 0.05


def test_rgb_color_gradient_is_chain_rule_of_dc_sh():
    """Gradients in RGB mode: dL/dc = dL/dbeta0 / Y00 of the matching DC-only SH
    scene, every other parameter's gradient as in that scene (the colour has no
    view dependence in either), and exactly zero on the 45 unused SH rows."""
    p, cam = tiny_scene(6, 67)
    c = np.random.default_rng(10).normal(0.0, 1.0, (3, p.shape[1]))
    p_rgb = p.copy()
    p_rgb[27:30] = c
    p_rgb[30:75] = np.random.default_rng(11).normal(0.0, 5.0, (45, p.shape[1]))
    p_sh = p.copy()
    p_sh[27:30] = c / Y00
    p_sh[30:75] = 0.0
    w = np.random.default_rng(12).normal(size=(3, cam.height, cam.width))
    g_rgb, _ = oracle.backward(p_rgb, cam, w, oracle.Settings(rgb_color=True), nthreads=1)
    g_sh, _ = oracle.backward(p_sh, cam, w, oracle.Settings(), nthreads=1)
    scale = np.abs(g_sh).max()
    assert np.all(g_rgb[30:75] == 0.0)
    assert np.abs(g_rgb[27:30] - g_sh[27:30] / Y00).max() <= 1e-10 * scale
    for r0, r1 in ((0, 27), (75, 76)):
        assert np.abs(g_rgb[r0:r1] - g_sh[r0:r1]).max() <= 1e-10 * scale


def test_rgb_color_gradient_matches_finite_differences():
    """dL/dc in RGB mode against FP64 central differences of the render."""
    n = 5
    p, cam = tiny_scene(n, 71)
    st = oracle.Settings(rgb_color=True, bg=(0.2, 0.1, 0.3))
    w = np.random.default_rng(13).normal(size=(3, cam.height, cam.width))

    def loss(pp):
        img, *_ = oracle.render(pp, cam, st, nthreads=1)
        return float((img * w).sum())

    g, _ = oracle.backward(p, cam, w, st, nthreads=1)
    for row in (27, 28, 29):
        for i in range(n):
            h = 1e-6
            pp = p.copy(); pp[row, i] += h
            pm = p.copy(); pm[row, i] -= h
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(g[row, i] - fd) <= 1e-6 * max(abs(fd), 1e-3)


# --------------------------------------------- the slice's direction-independent part
def test_static_part_reproduces_the_slice():
    """The cached quantities rebuild the slice: mu_cond = mu_p + K (d - mu_d),
    D = (d - mu_d)^T Sigma_d^-1 (d - mu_d), alpha_cond = alpha exp(-lambda D)
    and Sigma_cond equal the oracle's slice (pinned above against the precision
    form and the Woodbury identity) for arbitrary unit directions."""
    n = 200
    p = synth.make_scene(synth.workload("c2", n).scene)
    st = oracle.static_part(p)
    rng = np.random.default_rng(17)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    mu_c, sig, D, f, ac = oracle.slice_gaussians(p, d, 0.35)
    K = st[6:15].T.reshape(n, 3, 3)
    a = st[15:21].T
    A = np.stack([a[:, [0, 1, 2]], a[:, [1, 3, 4]], a[:, [2, 4, 5]]], axis=1)
    sc = st[0:6].T
    Sc = np.stack([sc[:, [0, 1, 2]], sc[:, [1, 3, 4]], sc[:, [2, 4, 5]]], axis=1)
    x = d - p[3:6].T
    assert np.abs(p[0:3].T + np.einsum("nij,nj->ni", K, x) - mu_c).max() < 1e-12
    Dc = np.einsum("ni,nij,nj->n", x, A, x)
    assert np.abs(Dc - D).max() <= 1e-12 * max(1.0, np.abs(D).max())
    assert np.abs(st[21] * np.exp(-0.35 * Dc) - ac).max() < 1e-12
    assert np.abs(Sc - sig).max() <= 1e-12 * np.abs(sig).max()
    assert np.all(np.linalg.eigvalsh(A) > 0)  # an inverse covariance
