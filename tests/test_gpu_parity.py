"""GPU parity: the HIP path (through its C ABI) against the FP64 oracle on the
same seeded inputs.

Bars (derived from float32 arithmetic against float64, see the design notes):
  * integer stage (tile counts, keys, order, ranges) bit-exact given the same
    float32 records;
  * records within the float32 error bounds the oracle's decision envelope
    assumes;
  * every pixel inside its decision envelope up to 1e-4 absolute (the
    definition's value itself where no threshold decision is undecided);
  * gradients within 1e-3 relative (norm per parameter group, and per element
    against a floor of 1e-2 of the group's largest), with the upstream
    gradient zeroed where an undecided decision could move a term.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from tests import _gpu as G

pytestmark = pytest.mark.gpu

PIX_TOL = G.PIX_TOL


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2410_04974_amd import lib
    lib()  # fails loudly when lib6dgs.so is missing
    yield


# ------------------------------------------------------------------ records
def _conic_metric_error(gpu, ref):
    """max |x^T (Q_gpu - Q) x| / x^T Q x over x: the conic's error in its own
    metric (the largest |eigenvalue| of Q^-1 (Q_gpu - Q))."""
    m = len(ref)
    Q = np.zeros((m, 2, 2))
    dQ = np.zeros((m, 2, 2))
    Q[:, 0, 0], Q[:, 0, 1], Q[:, 1, 0], Q[:, 1, 1] = ref[:, 0], ref[:, 1], ref[:, 1], ref[:, 2]
    g = gpu.astype(np.float64) - ref
    dQ[:, 0, 0], dQ[:, 0, 1], dQ[:, 1, 0], dQ[:, 1, 1] = g[:, 0], g[:, 1], g[:, 1], g[:, 2]
    return np.abs(np.linalg.eigvals(np.linalg.solve(Q, dQ))).max(axis=1)


@pytest.mark.parametrize("name,n,view", [("c0", None, 0), ("c1", None, 0), ("c2", None, 0), ("r1", None, 0),
                                         ("r2", None, 0), ("c4", None, 5)])
def test_records_match_oracle(name, n, view):
    """The GPU's float32 records against the FP64 ones at full size, and within
    the float32 error bounds that the oracle's decision envelope assumes (so
    the envelope covers every decision the GPU can take the other way)."""
    w, p = G.scene(name, n)
    cam = w.cameras[view]
    r, _, _ = G.render(p, [cam])
    rec, tiles = G.records(r)
    o = oracle.preprocess(p, cam)
    st = oracle.Settings()
    alive_o = o["alive"]
    binned = tiles > 0
    # an entry binned on one side only is one the envelope treats as near the cut
    one_side = binned ^ alive_o
    assert (o["near_cut"][one_side & ~alive_o] == 1).all()
    both = binned & alive_o
    _say(name, "binned", binned.sum(), "oracle alive", alive_o.sum(), "one side only", one_side.sum())
    assert both.sum() >= 0.999 * binned.sum()
    e = {}
    e["uv"] = max(np.abs(rec[both, G.REC_U] - o["u"][both]).max(), np.abs(rec[both, G.REC_V] - o["v"][both]).max())
    e["conic"] = _conic_metric_error(rec[both][:, [G.REC_QXX, G.REC_QXY, G.REC_QYY]], o["conic"][both]).max()
    e["alpha_c"] = G.rel_err(rec[both, G.REC_AC], o["alpha_cond"][both], 1e-30).max()
    e["rgb"] = np.abs(rec[both][:, [G.REC_R, G.REC_G, G.REC_B]] - o["rgb"][both]).max()
    e["depth"] = G.rel_err(rec[both, G.REC_DEPTH], o["depth"][both], 1e-30).max()
    # the extents are sqrt(q_max * Sigma2D_xx) with q_max = 2 ln(255 alpha_cond): compare the
    # q_max they imply (its absolute error, unlike the extent's relative one, stays bounded as
    # alpha_cond approaches 1/255)
    e["qmax_x"] = (np.abs(rec[both, G.REC_EX].astype(np.float64) ** 2 - o["ex"][both] ** 2) / o["cov2d"][both, 0]).max()
    e["qmax_y"] = (np.abs(rec[both, G.REC_EY].astype(np.float64) ** 2 - o["ey"][both] ** 2) / o["cov2d"][both, 2]).max()
    bounds = {"uv": st.uv_margin(cam), "conic": st.m_conic, "alpha_c": st.m_alpha, "depth": st.m_depth}
    _say(name, {k: f"{v:.2e}" + (f" (bound {bounds[k]:.1e})" if k in bounds else "") for k, v in e.items()})
    for k, b in bounds.items():
        assert e[k] <= b, (k, e[k], b)
    assert e["rgb"] < 1e-6
    assert max(e["qmax_x"], e["qmax_y"]) < 1e-4


# ------------------------------------------------------------ integer stage
def _random_records(n, cams, seed, ext=10.0):
    rng = np.random.default_rng(seed)
    E = n * len(cams)
    W = max(c.width for c in cams)
    H = max(c.height for c in cams)
    u = rng.uniform(-0.2 * W, 1.2 * W, E).astype(np.float32)
    v = rng.uniform(-0.2 * H, 1.2 * H, E).astype(np.float32)
    ex = rng.exponential(ext, E).astype(np.float32)
    ey = rng.exponential(ext, E).astype(np.float32)
    big = rng.random(E) < 0.002
    ex[big] *= 30
    ey[big] *= 30
    depth = rng.uniform(0.5, 8.0, E).astype(np.float32)
    ties = rng.random(E) < 0.3
    depth[ties] = np.float32(2.0)  # many exactly equal depths: order falls back to entry id
    alive = (rng.random(E) < 0.9).astype(np.int32)
    # some extents exactly on tile boundaries
    k = rng.random(E) < 0.05
    u[k] = np.float32(32.0) + ex[k]
    return u, v, ex, ey, depth, alive


@pytest.mark.parametrize("tile", [(16, 16), (32, 8), (8, 32)])
@pytest.mark.parametrize("case", ["one_view", "three_views", "empty", "one_octave", "one_tile"])
def test_binning_bit_exact(tile, case):
    """one_octave: every depth in [2, 4), so the depth keys' top byte is the
    same for all (that radix pass keeps the order and copies); one_tile: an
    image of one tile, every pair with the same key."""
    if case in ("one_view", "one_octave"):
        cams = [synth.default_camera(203, 157)]
        n = 5000
    elif case == "one_tile":
        cams = [synth.default_camera(tile[0], tile[1])]
        n = 3000
    elif case == "three_views":
        cams = [synth.default_camera(64, 64), synth.default_camera(400, 130), synth.default_camera(33, 517)]
        n = 3000
    else:
        cams = [synth.default_camera(100, 100)]
        n = 700
    u, v, ex, ey, depth, alive = _random_records(n, cams, seed=11)
    if case == "empty":
        alive[:] = 0
    if case == "one_octave":
        depth = (2.0 + (depth - 0.5) / 7.5 * 1.999).astype(np.float32)
        depth[::7] = np.float32(3.0)  # equal depths still fall back to entry order
    r = G.renderer(tile=tile)
    dev = [torch.from_numpy(a).to(G.DEV) for a in (u, v, ex, ey, depth, alive)]
    r.ctx.bin(n, cams, *dev)
    from paper_2410_04974_amd import _lib
    keys = r.ctx.export(_lib.EXPORT_KEYS)
    vals = r.ctx.export(_lib.EXPORT_VALUES)
    ranges = r.ctx.export(_lib.EXPORT_RANGES)
    tiles = r.ctx.export(_lib.EXPORT_TILES)
    ref = oracle.bin_records(u, v, ex, ey, depth, alive.astype(bool), n, cams, tile[0], tile[1])
    _say(case, tile, "pairs", len(ref["keys"]))
    assert np.array_equal(tiles, ref["tiles_touched"].astype(np.int32))
    assert np.array_equal(keys, ref["keys"])
    assert np.array_equal(vals, ref["values"].astype(np.int32))
    assert np.array_equal(ranges, ref["ranges"].astype(np.int32))


@pytest.mark.parametrize("case", ["c2_size", "sixteen_1080p_views"])
def test_binning_bit_exact_at_full_size(case):
    """The integer stage at the sizes the benchmarks run: ~300k entries giving
    several million pairs on one 800x800 view (a 12-bit tile id: two 6-bit
    passes), and 16 views of 1920x1080 (130k tiles: three passes), in both the
    growing and the fixed-capacity mode."""
    if case == "c2_size":
        cams, n, ext = [synth.default_camera(800, 800)], 300000, 30.0
    else:
        cams, n, ext = [synth.default_camera(1920, 1080)] * 16, 40000, 20.0
    u, v, ex, ey, depth, alive = _random_records(n, cams, seed=12, ext=ext)
    ref = oracle.bin_records(u, v, ex, ey, depth, alive.astype(bool), n, cams, 16, 16)
    P = len(ref["keys"])
    from paper_2410_04974_amd import _lib
    dev = [torch.from_numpy(a).to(G.DEV) for a in (u, v, ex, ey, depth, alive)]
    for cap in (0, P + 12345):
        r = G.renderer()
        r.configure(pair_capacity=cap)
        r.ctx.bin(n, cams, *dev)
        r.ctx.check()
        _say(case, "pairs", P, "capacity", cap)
        assert np.array_equal(r.ctx.export(_lib.EXPORT_KEYS), ref["keys"])
        assert np.array_equal(r.ctx.export(_lib.EXPORT_VALUES), ref["values"].astype(np.int32))
        assert np.array_equal(r.ctx.export(_lib.EXPORT_RANGES), ref["ranges"].astype(np.int32))


def test_pair_overflow_at_fixed_capacity_is_reported_and_renders_background():
    """A fixed pair capacity below the pair count: nothing is binned, so the
    forward renders the background alone (no pair list is read), check()
    reports the capacity error once, and a context with room for the pairs
    renders the image the growing mode renders."""
    from paper_2410_04974_amd import SixDGSError, _lib
    w, pn = G.scene("c1", 20000)
    cam = synth.default_camera(160, 128)
    p = G.to_dev(pn)
    bg = (0.25, 0.5, 0.75)
    grow = G.renderer(bg=bg)
    ref = grow.forward(p, [cam])[0]
    grow.ctx.check()
    P = grow.ctx.sizes()["pairs"]
    _say("pairs", P)
    assert P > 1000
    r = G.renderer(bg=bg, pair_capacity=P // 2)
    img = r.forward(p, [cam])[0]
    with pytest.raises(SixDGSError) as e:
        r.ctx.check()
    assert e.value.status == _lib.ERR_CAPACITY
    r.ctx.check()  # reported once
    want = torch.tensor(bg, device=G.DEV, dtype=torch.float32).view(3, 1, 1).expand_as(img)
    assert torch.equal(img, want)
    roomy = G.renderer(bg=bg, pair_capacity=P + 4096)
    img2 = roomy.forward(p, [cam])[0]
    roomy.ctx.check()
    assert torch.equal(img2, ref)


# ------------------------------------------------------------------ forward
@pytest.mark.parametrize("tile", [(16, 16), (32, 8)])
def test_forward_full_frame_c0(tile):
    w, p = G.scene("c0")
    cam = w.cameras[0]
    r, _, imgs = G.render(p, [cam], tile=tile, flags=1)
    from paper_2410_04974_amd import _lib
    T = r.ctx.export(_lib.EXPORT_T_FINAL).reshape(cam.height, cam.width)
    cnt = r.ctx.export(_lib.EXPORT_COUNTS).reshape(cam.height, cam.width)
    env = oracle.render_envelope(p, cam)
    G.check_envelope(imgs[0], T, env, f"c0 {tile}", _say)
    ok = ~env["ambiguous"]
    assert np.array_equal(cnt[ok], env["ncontrib"][ok])


def test_forward_ragged_multi_tile_scene_with_background():
    """Image sizes that are not tile multiples, a non-zero background and a
    scene dense enough to fill many tiles; every pixel checked."""
    w, p = G.scene("c1", 30000)
    cam = synth.default_camera(203, 150)
    st = oracle.Settings(bg=(0.25, 0.5, 1.0))
    r, _, imgs = G.render(p, [cam], bg=st.bg)
    from paper_2410_04974_amd import _lib
    T = r.ctx.export(_lib.EXPORT_T_FINAL).reshape(cam.height, cam.width)
    G.check_envelope(imgs[0], T, oracle.render_envelope(p, cam, st), "ragged", _say)


@pytest.mark.parametrize("name", ["c1", "c2", "r1", "r2"])
def test_forward_sampled_pixels_full_size(name):
    """Full-size workload, 4096 seeded pixels against the oracle, each inside
    its decision envelope."""
    w, p = G.scene(name)
    cam = w.cameras[0]
    r, _, imgs = G.render(p, [cam])
    from paper_2410_04974_amd import _lib
    T = r.ctx.export(_lib.EXPORT_T_FINAL)
    pix = synth.pixel_subset(cam.width, cam.height, 4096)
    env = oracle.render_envelope(p, cam, pixels=pix)
    img = imgs[0].reshape(3, -1)[:, pix]
    st = G.check_envelope(img, T[pix], env, name, _say)
    # a loosened check (an envelope wider than the bar) on a small minority only
    assert st["width_gt_tol_frac"] < 0.03


def test_forward_sampled_pixels_c4_view():
    """One 1920x1080 view of the 1M-Gaussian mixed scene (near Gaussians of the
    cube part, the widest depth range of the workloads)."""
    w, p = G.scene("c4")
    cam = w.cameras[5]
    r, _, imgs = G.render(p, [cam])
    from paper_2410_04974_amd import _lib
    T = r.ctx.export(_lib.EXPORT_T_FINAL)
    pix = synth.pixel_subset(cam.width, cam.height, 4096)
    env = oracle.render_envelope(p, cam, pixels=pix)
    st = G.check_envelope(imgs[0].reshape(3, -1)[:, pix], T[pix], env, "c4 view 5", _say)
    assert st["width_gt_tol_frac"] < 0.03


def test_forward_tile_shapes_bitwise_equal():
    """The image does not depend on the tile shape or batch depth."""
    w, p = G.scene("c1", 30000)
    cam = synth.default_camera(256, 192)
    outs = []
    for tile, batch in (((16, 16), 256), ((32, 8), 128), ((8, 32), 64), ((16, 16), 128)):
        _, _, imgs = G.render(p, [cam], tile=tile, batch=batch)
        outs.append(imgs[0])
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


# ----------------------------------------------------------------- backward
def _group_errors(g, ref):
    out = {}
    for nm, (a, b) in {"mu_p": (0, 3), "mu_d": (3, 6), "L": (6, 27), "sh": (27, 75), "opacity": (75, 76)}.items():
        den = np.linalg.norm(ref[a:b])
        out[nm] = np.linalg.norm(g[a:b] - ref[a:b]) / max(den, 1e-30)
    return out


@pytest.mark.parametrize("name,n,size", [("c1", 20000, (256, 256)), ("c2", 20000, (200, 160))])
def test_backward_matches_oracle_gradient(name, n, size):
    w, p = G.scene(name, n)
    cam = synth.default_camera(*size)
    env = oracle.render_envelope(p, cam)
    dl = synth.upstream_gradient([cam])[0].astype(np.float64)
    skip = G.grad_mask(env)
    dl[:, skip] = 0.0  # no gradient through pixels with an undecided threshold decision
    r, pt, _ = G.render(p, [cam])
    g = r.backward(pt, [torch.from_numpy(dl.astype(np.float32)).to(G.DEV)]).cpu().numpy().astype(np.float64)
    ref, _ = oracle.backward(p, cam, dl)
    errs = _group_errors(g, ref)
    _say(name, "pixels left out", f"{skip.mean():.4f}", "grad rel err per group", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v < 1e-3 for v in errs.values())


def _element_errors(g, ref):
    """Per-element error against 1e-3 max(|g*|, 1e-2 max|g*|) per parameter group."""
    out = {}
    for nm, (a, b) in {"mu_p": (0, 3), "mu_d": (3, 6), "L": (6, 27), "sh": (27, 75), "opacity": (75, 76)}.items():
        r = ref[a:b]
        bar = 1e-3 * np.maximum(np.abs(r), 1e-2 * np.abs(r).max())
        out[nm] = float((np.abs(g[a:b] - r) / bar).max())
    return out


@pytest.mark.parametrize("name", ["c2", "c1"])
def test_backward_full_size_sampled_pixels_match_oracle(name):
    """The benchmarked configuration at full size: 300k Gaussians (c2: strong
    spatial-direction coupling, L_dp raw N(0, 0.3)) at 800x800 with the
    automatic batch depth and chunk (128 / 128: heavy tiles span dozens of
    backward work items restarted from forward-saved state).  dL/dI is
    non-zero on the seeded sample of 4096 pixels only, and zero on those of
    them with any undecided threshold decision (the gradient there depends on
    which way float32 takes it); the 76-row gradient is compared with the
    oracle's analytic gradient of the same pixels, per group and per element."""
    w, p = G.scene(name)
    cam = w.cameras[0]
    pix = synth.pixel_subset(cam.width, cam.height, 4096)
    env = oracle.render_envelope(p, cam, pixels=pix)
    keep = ~G.grad_mask(env)
    rng = np.random.default_rng(synth.SEED_UPSTREAM)
    dsub = (rng.normal(0.0, 1.0, (len(pix), 3)) * keep[:, None]).astype(np.float32)
    dl = np.zeros((3, cam.height * cam.width), np.float32)
    dl[:, pix] = dsub.T
    r, pt, _ = G.render(p, [cam])
    sz = r.ctx.sizes()
    g = r.backward(pt, [torch.from_numpy(dl.reshape(3, cam.height, cam.width)).to(G.DEV)]).cpu().numpy()
    g = g.astype(np.float64)
    ref, _ = oracle.backward(p, cam, dsub.astype(np.float64), pixels=pix)
    errs = _group_errors(g, ref)
    el = _element_errors(g, ref)
    _say(name, "batch/chunk", sz["batch"], sz["chunk"], "pixels used", int(keep.sum()),
         "group", {k: f"{v:.1e}" for k, v in errs.items()}, "element / bar", {k: f"{v:.2f}" for k, v in el.items()})
    assert (sz["batch"], sz["chunk"]) == (128, 128)
    assert keep.sum() > 2048
    assert all(v < 1e-3 for v in errs.values())
    assert all(v <= 1.0 for v in el.values())


@pytest.mark.parametrize("name,batch", [("c1", 256), ("c1", 64), ("c1", 0), ("c2", 0)])
def test_backward_chunk_lengths_agree(name, batch):
    """The backward walks each tile's list in work items of `chunk` positions,
    restarted from state the forward saved; any chunk length gives the same
    gradient up to float32 rounding (c1 and c2 at full size: heavy tiles span
    many chunks).  batch 0: the automatic batch depth and chunk (128 / 128
    here), the configuration the training-step benchmark times; the oracle
    comparisons and the finite-difference check use it too."""
    w, pn = G.scene(name)
    cam = w.cameras[0]
    dl = torch.from_numpy(synth.upstream_gradient([cam])[0]).to(G.DEV)
    p = G.to_dev(pn)
    grads = {}
    for chunk in (batch, 1024, 16384):
        r = G.renderer(batch=batch, chunk=chunk)
        r.forward(p, [cam])
        grads[chunk] = r.backward(p, [dl]).cpu().numpy().astype(np.float64)
    ref = grads[16384]
    for chunk in (batch, 1024):
        errs = _group_errors(grads[chunk], ref)
        _say("batch", batch, "chunk", chunk, "vs one chunk per tile", {k: f"{v:.1e}" for k, v in errs.items()})
        assert all(v < 2e-5 for v in errs.values())


def test_second_backward_of_one_forward_repeats_the_gradient():
    """The forward clears the screen-space gradient accumulators for the
    backward that follows; a second backward of the same forward clears them
    itself, so it returns the same gradient (up to the order of float atomics)."""
    w, pn = G.scene("c1", 20000)
    cam = synth.default_camera(160, 128)
    r, p, _ = G.render(pn, [cam])
    dl = torch.from_numpy(synth.upstream_gradient([cam])[0]).to(G.DEV)
    g1 = r.backward(p, [dl]).cpu().numpy().astype(np.float64)
    g2 = r.backward(p, [dl]).cpu().numpy().astype(np.float64)
    scale = np.abs(g1).max()
    assert scale > 0
    assert np.abs(g1 - g2).max() <= 1e-5 * scale


def test_backward_ignores_lds_left_by_earlier_kernels():
    """The backward reads its staged records through per-wavefront slot lists;
    the slots past a list's end hold whatever an earlier kernel left in LDS.
    With reductions over NaN run between the forward and the backward (their
    partial sums pass through LDS), the gradient stays finite and equal to the
    one computed without them (up to the order of float atomics)."""
    w, pn = G.scene("c1")
    cam = w.cameras[0]
    p = G.to_dev(pn)
    dl = torch.from_numpy(synth.upstream_gradient([cam])[0]).to(G.DEV)
    r = G.renderer(chunk=16384)
    r.forward(p, [cam])
    g1 = r.backward(p, [dl]).cpu().numpy().astype(np.float64)
    poison = torch.full((1 << 24,), float("nan"), device=G.DEV)
    r.forward(p, [cam])
    for _ in range(4):
        poison.sum()
        torch.softmax(poison.view(-1, 4096), dim=1)
        torch.cumsum(poison.view(-1, 4096), dim=1)
    g2 = r.backward(p, [dl]).cpu().numpy().astype(np.float64)
    assert np.isfinite(g2).all()
    scale = np.abs(g1).max()
    assert np.abs(g1 - g2).max() <= 1e-5 * scale
