"""Pins of the oracle's decision envelope (``oracle.render_envelope``).

The compositing walk of Sec. 4.4 (the 3D Gaussian splatting rasteriser) takes
threshold decisions -- skip a Gaussian with alpha below 1/255, stop before the
transmittance falls below 1e-4, order Gaussians by depth -- that a float32
renderer may legitimately take the other way when its records differ from the
float64 ones within float32 error bounds.  The envelope is the range of the
pixel over every combination of such outcomes.  These tests fix it against
hand-computed two- and one-Gaussian pixels and check, by moving whole scenes'
records within the stated bounds, that no pixel can leave its envelope: the
claim every GPU parity test relies on.
"""
import math

import numpy as np
import pytest

import oracle
import synth

AMIN = 1.0 / 255.0


def rec(u, v, sigma, ac, rgb, depth, alive=1.0):
    """One isotropic record (conic 1 / sigma^2) as oracle.render_records takes it."""
    q = 1.0 / sigma ** 2
    return [u, v, q, 0.0, q, ac, *rgb, depth, alive]


def one_pixel(records, settings=None, W=41, H=41, px=20, py=20):
    cam = synth.default_camera(W, H)
    st = settings or oracle.Settings(m_uv=1e-4)
    return oracle.render_records(np.array(records, np.float64), cam, st, pixels=[py * W + px])


def offset_for_alpha(sigma, ac, a):
    """Distance from the mean at which ac exp(-r^2 / (2 sigma^2)) equals a."""
    return sigma * math.sqrt(2.0 * math.log(ac / a))


@pytest.mark.parametrize("side", [-1.0, 1.0])
def test_alpha_just_at_the_cut_is_ambiguous_with_both_outcomes(side):
    """A Gaussian whose alpha at the pixel is 1/255 (1 +- 1e-7): far inside any
    float32 error, so both the skip and the take are possible and the envelope
    spans the background and the composite."""
    sigma, ac, rgb = 3.0, 0.6, (0.9, 0.2, 0.5)
    r = offset_for_alpha(sigma, ac, AMIN * (1.0 + side * 1e-7))
    st = oracle.Settings(m_uv=1e-4, bg=(0.1, 0.3, 0.7))
    e = one_pixel([rec(20.5 - r, 20.5, sigma, ac, rgb, 3.0)], st)
    a = ac * math.exp(-0.5 * r * r / sigma ** 2)
    assert e["ambiguous"][0] and e["leaves"][0] == 2
    skip = np.array(st.bg)
    take = np.array(rgb) * a + np.array(st.bg) * (1 - a)
    assert np.allclose(e["lo"][0], np.minimum(skip, take), atol=1e-15)
    assert np.allclose(e["hi"][0], np.maximum(skip, take), atol=1e-15)
    assert e["T_lo"][0] == pytest.approx(1 - a, abs=1e-15) and e["T_hi"][0] == 1.0
    # the definition takes it exactly when alpha >= 1/255
    assert e["ncontrib"][0] == (1 if side > 0 else 0)
    assert e["impact"][0] == pytest.approx(a, rel=1e-12)


def test_alpha_far_from_the_cut_is_not_ambiguous():
    sigma, ac, rgb = 3.0, 0.6, (0.9, 0.2, 0.5)
    for target in (AMIN * 1.01, AMIN * 0.99, 0.3):
        r = offset_for_alpha(sigma, ac, target)
        e = one_pixel([rec(20.5 - r, 20.5, sigma, ac, rgb, 3.0)])
        assert not e["ambiguous"][0] and e["leaves"][0] == 1 and e["impact"][0] == 0.0
        assert np.array_equal(e["lo"][0], e["color"][0]) and np.array_equal(e["hi"][0], e["color"][0])


def test_margin_of_the_cut_scales_with_the_position_error():
    """The band of alpha around 1/255 that is ambiguous widens with the mean's
    error bound m_uv: the same pixel is decided at m_uv = 1e-6 px and undecided
    at 1e-2 px (alpha there is 1/255 (1 + 1e-3))."""
    sigma, ac = 3.0, 0.6
    r = offset_for_alpha(sigma, ac, AMIN * (1.0 + 1e-3))
    g = [rec(20.5 - r, 20.5, sigma, ac, (0.5, 0.5, 0.5), 3.0)]
    assert not one_pixel(g, oracle.Settings(m_uv=1e-6))["ambiguous"][0]
    assert one_pixel(g, oracle.Settings(m_uv=1e-2))["ambiguous"][0]


def test_near_cut_gaussian_that_the_definition_culls_is_a_possible_take():
    """alpha_cond just below 1/255: the definition culls the Gaussian, but a
    float32 alpha_cond may reach the cut, so at its centre the take is an
    outcome too."""
    ac = AMIN * (1.0 - 1e-6)
    e = one_pixel([rec(20.5, 20.5, 3.0, ac, (1.0, 1.0, 1.0), 3.0)])
    assert e["ncontrib"][0] == 0 and e["ambiguous"][0]
    assert e["hi"][0][0] == pytest.approx(ac, rel=1e-12) and e["lo"][0][0] == 0.0


def test_stop_at_t_min_is_ambiguous_within_rounding_and_decided_outside():
    """Three opaque Gaussians: T after the third is 1e-4 (1 +- eps).  For eps far
    below float32 rounding of the transmittance both stop and go are possible;
    for eps = 1e-2 the decision is fixed.  (Between the two the margin is set by
    alpha_cond's error: at a = 0.98 its relative error 3e-5 makes 1 - a
    uncertain by 49 times that, 1.5e-3.)"""
    cs = [np.array(c) for c in ((0.2, 0.4, 0.6), (0.9, 0.1, 0.3), (0.5, 0.7, 0.1))]
    for eps, amb in ((1e-9, True), (-1e-9, True), (1e-3, True), (1e-2, False), (-1e-2, False)):
        al = [0.98, 0.95, 0.9 - 0.1 * eps]  # T: 0.02, 1e-3, 1e-4 (1 + eps)
        g = [rec(20.5, 20.5, 5.0, al[k], cs[k], 2.0 + k) for k in range(3)]
        e = one_pixel(g)
        assert bool(e["ambiguous"][0]) == amb, eps
        T2 = (1 - al[0]) * (1 - al[1])
        stop = cs[0] * al[0] + cs[1] * al[1] * (1 - al[0])
        go = stop + cs[2] * al[2] * T2
        if amb:
            assert np.allclose(e["lo"][0], np.minimum(stop, go), atol=1e-15)
            assert np.allclose(e["hi"][0], np.maximum(stop, go), atol=1e-15)
            assert e["T_hi"][0] == pytest.approx(T2, rel=1e-12)
        else:
            want = go if eps > 0 else stop
            assert np.allclose(e["lo"][0], want, atol=1e-15) and np.allclose(e["hi"][0], want, atol=1e-15)


def test_nearly_equal_depths_take_both_orders():
    """Two overlapping Gaussians whose depths differ by 1e-8 relative: their
    order is undecided, the envelope holds both composites; 1e-3 apart: decided."""
    c1, c2 = np.array([1.0, 0.0, 0.2]), np.array([0.0, 1.0, 0.2])
    a1, a2 = 0.5, 0.7
    front = c1 * a1 + c2 * a2 * (1 - a1)
    back = c2 * a2 + c1 * a1 * (1 - a2)
    for dz, amb in ((1e-8, True), (1e-3, False)):
        g = [rec(20.5, 20.5, 5.0, a1, c1, 3.0), rec(20.5, 20.5, 5.0, a2, c2, 3.0 * (1 + dz))]
        e = one_pixel(g)
        assert bool(e["ambiguous"][0]) == amb
        if amb:
            assert np.allclose(e["lo"][0], np.minimum(front, back), atol=1e-15)
            assert np.allclose(e["hi"][0], np.maximum(front, back), atol=1e-15)
            assert e["impact"][0] == pytest.approx(a1 * a2, rel=1e-12)
            assert e["T_lo"][0] == pytest.approx((1 - a1) * (1 - a2), rel=1e-12)
        else:
            assert np.allclose(e["lo"][0], front, atol=1e-15) and np.allclose(e["hi"][0], front, atol=1e-15)


def test_three_way_tie_takes_all_six_orders():
    cs = [np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])]
    al = [0.3, 0.5, 0.6]
    g = [rec(20.5, 20.5, 5.0, al[k], cs[k], 3.0 * (1 + 1e-9 * k)) for k in range(3)]
    e = one_pixel(g)
    import itertools
    outs = []
    for perm in itertools.permutations(range(3)):
        T, C = 1.0, np.zeros(3)
        for k in perm:
            C += cs[k] * al[k] * T
            T *= 1 - al[k]
        outs.append(C)
    outs = np.array(outs)
    assert np.allclose(e["lo"][0], outs.min(axis=0), atol=1e-15)
    assert np.allclose(e["hi"][0], outs.max(axis=0), atol=1e-15)


def test_unambiguous_pixels_have_the_definition_as_their_envelope():
    w, p = synth.workload("c1", n_override=20000), None
    p = synth.make_scene(w.scene)
    cam = synth.default_camera(120, 96)
    e = oracle.render_envelope(p, cam, nthreads=4)
    c, T, n = oracle.render_plain(p, cam, nthreads=4)
    assert np.array_equal(e["color"], c) and np.array_equal(e["T"], T) and np.array_equal(e["ncontrib"], n)
    # merged outcome states keep one of several products equal up to rounding
    assert (e["lo"] <= c + 1e-12).all() and (e["hi"] >= c - 1e-12).all()
    ok = ~e["ambiguous"]
    assert ok.mean() > 0.5
    assert np.array_equal(e["lo"][:, ok], c[:, ok]) and np.array_equal(e["hi"][:, ok], c[:, ok])
    assert np.array_equal(e["T_lo"][ok], T[ok]) and np.array_equal(e["T_hi"][ok], T[ok])
    assert not e["unresolved"].any() and e["near_z"] == 0


# ----------------------------------------------- records moved within the bounds
def _moved(records, st, cam, rng, scale=1.0):
    """Every field moved within its error bound (times ``scale``): the mean by up
    to m_uv per axis, the conic by E = Q^1/2 S Q^1/2 with |S| <= m_conic (its
    error in its own metric), alpha_cond and depth by their relative bounds.
    Half of the draws sit at the bounds' extremes."""
    r = records.copy()
    m = len(r)
    def draw(k):
        x = rng.uniform(-1.0, 1.0, k)
        ext = rng.random(k) < 0.5
        x[ext] = np.sign(x[ext])
        return x * scale
    uv = st.uv_margin(cam)
    r[:, 0] += uv * draw(m)
    r[:, 1] += uv * draw(m)
    Q = np.zeros((m, 2, 2))
    Q[:, 0, 0], Q[:, 0, 1], Q[:, 1, 0], Q[:, 1, 1] = r[:, 2], r[:, 3], r[:, 3], r[:, 4]
    lam, V = np.linalg.eigh(Q)
    half = V * np.sqrt(np.maximum(lam, 0.0))[:, None, :] @ np.transpose(V, (0, 2, 1))
    th = rng.uniform(0, np.pi, m)
    Rt = np.stack([np.stack([np.cos(th), -np.sin(th)], 1), np.stack([np.sin(th), np.cos(th)], 1)], 1)
    S = Rt @ (np.eye(2) * (st.m_conic * np.stack([draw(m), draw(m)], 1))[:, :, None]) @ np.transpose(Rt, (0, 2, 1))
    E = half @ S @ half
    r[:, 2] += E[:, 0, 0]
    r[:, 3] += 0.5 * (E[:, 0, 1] + E[:, 1, 0])
    r[:, 4] += E[:, 1, 1]
    r[:, 5] *= 1.0 + st.m_alpha * draw(m)
    r[:, 9] *= 1.0 + st.m_depth * draw(m)
    return r


def _outside(e, moved, tol):
    c = moved["color"]
    out = np.maximum(e["lo"] - c, c - e["hi"]).max(axis=1)
    tout = np.maximum(e["T_lo"] - moved["T"], moved["T"] - e["T_hi"])
    return np.maximum(out, tout)


@pytest.mark.parametrize("name,n,size", [("c2", 40000, (160, 128)), ("c1", 30000, (200, 150)), ("r1", None, (176, 176))])
def test_records_moved_within_the_bounds_stay_inside_the_envelope(name, n, size):
    """The envelope's contract: records moved anywhere within the stated float32
    bounds render every pixel inside the envelope of the unmoved records, up to
    the 1e-4 bar that covers the continuous part of the change (the pixel tests
    use the same bar).  Several independent moves, half of each at the bounds'
    extremes; the moves do flip decisions (some pixels leave the unmoved value
    by far more than the bar) and every such pixel is one the envelope marks."""
    w = synth.workload(name, n_override=n)
    p = synth.make_scene(w.scene)
    cam = synth.default_camera(*size)
    st = oracle.Settings(bg=(0.2, 0.5, 0.8))
    base = oracle.records_of(p, cam, st)
    e = oracle.render_records(base, cam, st, nthreads=8)
    e = {k: (v.reshape(v.shape[0], -1).T if v.ndim == 3 else v.reshape(-1)) if isinstance(v, np.ndarray) else v
         for k, v in e.items()}
    rng = np.random.default_rng(7)
    flipped = 0
    for _ in range(3):
        mv = oracle.render_records(_moved(base, st, cam, rng), cam, st, nthreads=8, envelope=False)
        mv = {k: (v.reshape(v.shape[0], -1).T if v.ndim == 3 else v.reshape(-1)) if isinstance(v, np.ndarray) else v
              for k, v in mv.items()}
        assert _outside(e, mv, 1e-4).max() <= 1e-4
        jump = np.abs(mv["color"] - e["color"]).max(axis=1) > 1e-3
        assert not (jump & ~e["ambiguous"]).any()
        flipped += int(jump.sum())
    assert flipped > 0  # the moves did reach decisions


def test_an_envelope_with_too_small_bounds_misses_flips():
    """The same check with the envelope built for bounds 50 times smaller than
    the moves: some moved pixels land outside it, so the check above has teeth."""
    w = synth.workload("c2", n_override=40000)
    p = synth.make_scene(w.scene)
    cam = synth.default_camera(160, 128)
    st = oracle.Settings(bg=(0.2, 0.5, 0.8))
    small = oracle.Settings(bg=st.bg, m_uv=st.uv_margin(cam) / 50, m_conic=st.m_conic / 50,
                            m_alpha=st.m_alpha / 50, m_depth=st.m_depth / 50, m_eval=st.m_eval / 50)
    base = oracle.records_of(p, cam, st)
    flat = lambda d: {k: (v.reshape(v.shape[0], -1).T if v.ndim == 3 else v.reshape(-1))
                      if isinstance(v, np.ndarray) else v for k, v in d.items()}
    e = flat(oracle.render_records(base, cam, small, nthreads=8))
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(3):
        mv = flat(oracle.render_records(_moved(base, st, cam, rng), cam, st, nthreads=8, envelope=False))
        worst = max(worst, _outside(e, mv, 1e-4).max())
    assert worst > 1e-3
