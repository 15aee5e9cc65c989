"""The C ABI library loads on the host and exports every entry point its header
declares; argument checks that need no device run here too."""
import ctypes
import os
import re

import numpy as np

from paper_2410_04974_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "sixdgs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sixdgs_\w+)\s*\(", txt)))


def test_header_declares_the_binding_surface():
    decl = declared_functions()
    assert decl == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_default_settings_on_host():
    s = _lib.default_settings()
    assert abs(s.lambda_opa - 0.35) < 1e-7 and abs(s.z_near - 0.2) < 1e-7
    assert (s.tile_w, s.tile_h, s.batch, s.pair_capacity, s.chunk) == (16, 16, 0, 0, 0)  # 0: automatic


def test_adam_rejects_bad_arguments_before_any_launch():
    L = _lib.lib()
    lr = (ctypes.c_float * 6)(*([1e-3] * 6))
    # step 0 and beta out of range are refused without touching a device
    assert L.sixdgs_adam(None, None, None, None, 0, lr, 0.9, 0.999, 1e-15, 0, None) == _lib.ERR_INVALID_ARG
    assert L.sixdgs_adam(None, None, None, None, 0, lr, 1.5, 0.999, 1e-15, 1, None) == _lib.ERR_INVALID_ARG
    assert L.sixdgs_adam(None, None, None, None, 5, lr, 0.9, 0.999, 1e-15, 1, None) == _lib.ERR_INVALID_ARG


def test_create_rejects_unsupported_settings():
    L = _lib.lib()
    h = ctypes.c_void_p()
    for kw in ({"tile_w": 16, "tile_h": 8}, {"batch": 100}, {"batch": 32}, {"lambda_opa": 1.5}, {"z_near": 0.0},
               {"pair_capacity": -1}, {"tile_w": 32, "tile_h": 16}, {"pair_capacity": 1 << 30},
               {"batch": 256, "chunk": 128}, {"chunk": 32}, {"chunk": 1536}, {"chunk": 32768}, {"batch": -1},
               {"flags": 8}, {"flags": _lib.FLAG_DEBUG | 16}):
        s = _lib.default_settings(**kw)
        assert L.sixdgs_create(ctypes.byref(h), ctypes.byref(s)) == _lib.ERR_INVALID_ARG
        assert not h.value


def test_every_documented_flag_passes_the_settings_check():
    """Valid settings get past the checks (on a host without a device the
    context then fails at its first HIP call, not as an argument error)."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    for f in (_lib.FLAG_COUNTS, _lib.FLAG_RGB_COLOR, _lib.FLAG_DEBUG,
              _lib.FLAG_COUNTS | _lib.FLAG_RGB_COLOR | _lib.FLAG_DEBUG):
        s = _lib.default_settings(flags=f, chunk=64, batch=64)
        rc = L.sixdgs_create(ctypes.byref(h), ctypes.byref(s))
        assert rc != _lib.ERR_INVALID_ARG, f
        if rc == _lib.OK:
            L.sixdgs_destroy(h)


def test_l1_noalloc_rejects_bad_arguments_on_host():
    """The allocation-free L1 loss refuses bad arguments before touching a device."""
    L = _lib.lib()
    n1 = (ctypes.c_int64 * 1)(48)
    arr = (ctypes.c_void_p * 1)(None)
    assert L.sixdgs_l1_loss_noalloc(0, arr, arr, n1, arr, None, None) == _lib.ERR_INVALID_ARG
    assert L.sixdgs_l1_loss_noalloc(_lib.MAX_VIEWS + 1, arr, arr, n1, arr, None, None) == _lib.ERR_INVALID_ARG
    assert L.sixdgs_l1_loss_noalloc(1, arr, arr, n1, arr, None, None) == _lib.ERR_INVALID_ARG
