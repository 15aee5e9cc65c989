"""GPU: the allocation-free L1 loss (sixdgs_l1_loss_noalloc, fixed per-device
scratch) against sixdgs_l1_loss (context-owned scratch) and the FP64 oracle,
on two calls in a row -- the second smaller, so the scratch holds the first
call's partial sums when it starts."""
import numpy as np
import pytest
import torch

import oracle
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def _inputs(shapes, seed):
    rng = np.random.default_rng(seed)
    imgs = [rng.random(s).astype(np.float32) for s in shapes]
    tgts = [np.clip(a + rng.normal(0, 0.2, a.shape), 0, 1).astype(np.float32) for a in imgs]
    return imgs, tgts


def test_l1_noalloc_matches_l1_with_context_on_two_calls():
    from paper_2410_04974_amd import _lib
    ctx = _lib.Context()
    calls = [
        # 16 views, the largest call: 1024 partial sums for the 1080p view, many for the rest
        [(3, 1080, 1920)] + [(3, 64 + 9 * k, 80 + 7 * k) for k in range(15)],
        # then a smaller call: two ragged views, a handful of partial sums
        [(3, 37, 53), (3, 5, 7)],
    ]
    for shapes, seed in zip(calls, (1, 2)):
        imgs, tgts = _inputs(shapes, seed)
        I = [torch.from_numpy(a).to(G.DEV) for a in imgs]
        T = [torch.from_numpy(b).to(G.DEV) for b in tgts]
        g_ctx = [torch.full_like(a, 9.0) for a in I]
        g_na = [torch.full_like(a, 9.0) for a in I]
        l_ctx = torch.full((1,), 9.0, device=G.DEV)
        l_na = torch.full((1,), 9.0, device=G.DEV)
        ctx.l1_loss(I, T, g_ctx, l_ctx)
        _lib.l1_loss_noalloc(I, T, g_na, l_na)
        torch.cuda.synchronize()
        # the same kernels over the same partial-sum layout: bit-identical
        assert torch.equal(l_na, l_ctx)
        for a, b in zip(g_na, g_ctx):
            assert torch.equal(a, b)
        # and the definition (FP64): mean |I - I*| and sign(I - I*) / count
        ref_loss, ref_g = oracle.l1_loss(imgs, tgts)
        print("noalloc call", len(shapes), "images: loss", float(l_na), "oracle", ref_loss, flush=True)
        assert abs(float(l_na) - ref_loss) <= 1e-6 * max(1.0, abs(ref_loss))
        for a, b in zip(g_na, ref_g):
            assert np.array_equal(a.cpu().numpy(), b.astype(np.float32))


def test_l1_noalloc_rejects_bad_arguments():
    import ctypes
    from paper_2410_04974_amd import _lib
    a = torch.zeros((3, 4, 4), device=G.DEV)
    loss = torch.zeros(1, device=G.DEV)
    P = _lib._ptrs
    n1 = (ctypes.c_int64 * 1)(a.numel())
    L = _lib.lib()
    s = ctypes.c_void_p(_lib._stream(None))
    assert L.sixdgs_l1_loss_noalloc(0, P([a]), P([a]), n1, P([a]), ctypes.c_void_p(loss.data_ptr()), s) == _lib.ERR_INVALID_ARG
    assert L.sixdgs_l1_loss_noalloc(_lib.MAX_VIEWS + 1, P([a] * 17), P([a] * 17), (ctypes.c_int64 * 17)(*[48] * 17),
                                    P([a] * 17), ctypes.c_void_p(loss.data_ptr()), s) == _lib.ERR_INVALID_ARG
    assert L.sixdgs_l1_loss_noalloc(1, P([a]), P([a]), (ctypes.c_int64 * 1)(0), P([a]), ctypes.c_void_p(loss.data_ptr()), s) == _lib.ERR_INVALID_ARG
    assert L.sixdgs_l1_loss_noalloc(1, P([a]), None, n1, P([a]), ctypes.c_void_p(loss.data_ptr()), s) == _lib.ERR_INVALID_ARG
    assert L.sixdgs_l1_loss_noalloc(1, P([a]), P([a]), n1, P([a]), None, s) == _lib.ERR_INVALID_ARG
