"""The debug mode (SIXDGS_FLAG_DEBUG) on the GPU: every workspace buffer
carries guards and every call is followed by the guard and binning checks.
The renders and gradients are those of the normal mode, the checks pass on the
workloads' shapes (heavy tiles with chunk restarts, several uneven views, a
caller-given binning, a training step), and a write placed just outside a
buffer (from the host, with hipMemcpy: no kernel goes out of bounds) is
reported with the buffer's name.  Also the forward's run-to-run determinism
and the spread of the backward's atomically accumulated gradient."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[debug]", *a, flush=True)


def _lib():
    from paper_2410_04974_amd import _lib
    return _lib


def _run(p, cams, dls, debug, **kw):
    """Forward + backward on a fresh renderer; images, T_final, last and the gradient."""
    L = _lib()
    r = G.renderer(flags=L.FLAG_DEBUG if debug else 0, **kw)
    imgs = r.forward(p, cams)
    out = {"imgs": [i.clone() for i in imgs], "T": r.ctx.export(L.EXPORT_T_FINAL),
           "last": r.ctx.export(L.EXPORT_LAST), "sizes": r.ctx.sizes()}
    g = r.backward(p, dls)
    torch.cuda.synchronize()
    out["grad"] = g.clone()
    return out


def _spread(a, b):
    return float((a - b).abs().max() / a.abs().max())


@pytest.mark.parametrize("case", ["c2_heavy_tiles", "three_uneven_views"])
def test_debug_mode_passes_its_checks_and_matches_the_normal_mode(case):
    if case == "c2_heavy_tiles":
        # the benchmarked recipe on a small frame: runs of hundreds of pairs per
        # tile, walked by the backward in 64-long chunks
        w, pn = G.scene("c2", 40000)
        cams = [synth.default_camera(256, 192)]
        kw = dict(chunk=64, batch=64)
    else:
        w, pn = G.scene("c3", 20000)
        cams = [synth.default_camera(96, 80), synth.default_camera(200, 40), synth.default_camera(33, 130)]
        kw = {}
    p = G.to_dev(pn)
    dls = [torch.from_numpy(d).to(G.DEV) for d in synth.upstream_gradient(cams)]
    normal = _run(p, cams, dls, False, **kw)
    again = _run(p, cams, dls, False, **kw)
    debug = _run(p, cams, dls, True, **kw)
    _say(case, normal["sizes"])
    # the forward is deterministic, and the guards change nothing in it
    for o in (again, debug):
        for a, b in zip(normal["imgs"], o["imgs"]):
            assert torch.equal(a, b)
        assert np.array_equal(normal["T"], o["T"]) and np.array_equal(normal["last"], o["last"])
    # the backward adds screen-space gradients with float atomics: the order
    # (and so the rounding) varies from run to run; report the spread
    s_runs, s_debug = _spread(normal["grad"], again["grad"]), _spread(normal["grad"], debug["grad"])
    _say(case, f"gradient spread run-to-run {s_runs:.2e}, debug vs normal {s_debug:.2e}")
    assert s_runs < 1e-5 and s_debug < 1e-5


def test_debug_mode_checks_a_caller_given_binning():
    from tests.test_gpu_parity import _random_records
    L = _lib()
    cams = [synth.default_camera(64, 64), synth.default_camera(400, 130), synth.default_camera(33, 517)]
    n = 3000
    u, v, ex, ey, depth, alive = _random_records(n, cams, seed=11)
    depth[::7] = depth[0]  # equal depths: the check's tie order by entry id
    r = G.renderer(flags=L.FLAG_DEBUG)
    dev = [torch.from_numpy(a).to(G.DEV) for a in (u, v, ex, ey, depth, alive)]
    r.ctx.bin(n, cams, *dev)  # raises on a failed check
    r.ctx.check()
    _say("caller binning", r.ctx.sizes())


def test_debug_mode_training_steps():
    """Forward, L1 loss, backward and Adam through the trainer, three steps
    (the second with Adam fused into the preprocess backward)."""
    from paper_2410_04974_amd import Trainer
    L = _lib()
    w, pn = G.scene("c2", 20000)
    cam = synth.default_camera(160, 128)
    target = G.renderer().forward(G.to_dev(pn + 0.01), [cam])[0].clone()
    r = G.renderer(flags=L.FLAG_DEBUG)
    tr = Trainer(G.to_dev(pn), r)
    losses = [float(tr.step([cam], [target], fused=k == 1)) for k in range(3)]
    r.ctx.check()
    _say("losses", losses)
    assert all(np.isfinite(losses))


def _hip():
    return ctypes.CDLL("libamdhip64.so")


@pytest.mark.parametrize("where", ["past the end", "before the start"])
def test_a_write_outside_a_buffer_is_reported_with_its_name(where):
    L = _lib()
    w, pn = G.scene("c0", 500)
    p = G.to_dev(pn)
    cam = synth.default_camera(64, 48)
    r = G.renderer(flags=L.FLAG_DEBUG)
    r.forward(p, [cam])
    r.ctx.check()
    ptr, nbytes = ctypes.c_void_p(), ctypes.c_int64()
    assert L.lib().sixdgs_debug_buffer(r.ctx._h, b"ranges", ctypes.byref(ptr), ctypes.byref(nbytes)) == L.OK
    assert nbytes.value >= 8
    # 4 bytes inside the guard: the first past the end, or the last before the start
    dst = ptr.value + nbytes.value if where == "past the end" else ptr.value - 4
    word = ctypes.c_uint32(0x12345678)
    torch.cuda.synchronize()
    assert _hip().hipMemcpy(ctypes.c_void_p(dst), ctypes.byref(word), ctypes.c_size_t(4), 1) == 0
    rc = L.lib().sixdgs_check(r.ctx._h)
    msg = L.lib().sixdgs_last_error(r.ctx._h).decode()
    _say(where, msg)
    assert rc == L.ERR_DEBUG
    assert "ranges" in msg and ("past its end" if where == "past the end" else "before its start") in msg


def test_debug_buffer_lookup_errors_and_toggling_the_mode():
    L = _lib()
    w, pn = G.scene("c0", 300)
    p = G.to_dev(pn)
    cam = synth.default_camera(32, 32)
    ptr, nbytes = ctypes.c_void_p(), ctypes.c_int64()
    r = G.renderer()
    r.forward(p, [cam])
    assert L.lib().sixdgs_debug_buffer(r.ctx._h, b"ranges", ctypes.byref(ptr), ctypes.byref(nbytes)) == L.ERR_STATE
    # turning the mode on frees the workspace: the forward's state is gone
    r.configure(flags=L.FLAG_DEBUG)
    with pytest.raises(L.SixDGSError):
        r.ctx.backward(p, [torch.ones(3, 32, 32, device=G.DEV)], torch.zeros_like(p))
    assert L.lib().sixdgs_debug_buffer(r.ctx._h, b"no such buffer", ctypes.byref(ptr),
                                       ctypes.byref(nbytes)) == L.ERR_INVALID_ARG
    assert L.lib().sixdgs_debug_buffer(r.ctx._h, b"ranges", ctypes.byref(ptr), ctypes.byref(nbytes)) == L.ERR_STATE
    img_dbg = r.forward(p, [cam])[0].clone()
    assert L.lib().sixdgs_debug_buffer(r.ctx._h, b"ranges", ctypes.byref(ptr), ctypes.byref(nbytes)) == L.OK
    # and off again: the same image
    r.configure(flags=0)
    img = r.forward(p, [cam])[0]
    torch.cuda.synchronize()
    assert torch.equal(img, img_dbg)
