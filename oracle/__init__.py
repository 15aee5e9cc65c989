"""FP64 CPU oracle for the 6DGS renderer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2410_04974_amd``) and neither imports the other; the only common input
is the seeded generator module ``synth``.

Pieces:

* ``liboracle6dgs.so`` (``oracle6dgs.c``): the brute-force renderer, its
  analytic backward, the slice and the SH basis, all in double precision.
* ``binning``: the integer stage (tile rectangles, (tile, depth) keys, stable
  sort, per-tile ranges) as its plain definition in numpy, taking its decisions
  in float32 as the GPU does.
* ``l1_loss`` and ``adam_step``: textbook definitions in float64.

Readings of the paper where it is silent or ambiguous are listed in the module
docstring of ``oracle6dgs.c`` and in the project's design notes.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(closed forms, library routines, finite differences, brute force).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle6dgs.c")
_LIB = os.path.join(_HERE, "liboracle6dgs.so")

NROWS = 76
NREC = 38
NG2D = 9
FIELDS = {
    "alive": (0, 1), "mu_cond": (1, 3), "sigma_cond": (4, 6), "alpha": (10, 1), "f": (11, 1),
    "D": (12, 1), "alpha_cond": (13, 1), "rgb": (14, 3), "p": (17, 3), "depth": (20, 1),
    "u": (21, 1), "v": (22, 1), "cov2d": (23, 3), "conic": (26, 3), "ex": (29, 1), "ey": (30, 1),
    "dir": (31, 3), "sh_dir": (34, 3), "near_cut": (37, 1),
}
ENV_AMBIGUOUS, ENV_KINK, ENV_UNRESOLVED = 1, 2, 4


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (double precision, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cam(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int64), ("height", ctypes.c_int64)]


class _Set(ctypes.Structure):
    _fields_ = [("lambda_opa", ctypes.c_double), ("z_near", ctypes.c_double), ("bg", ctypes.c_double * 3),
                ("jac_guard", ctypes.c_double), ("dilation", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("t_min", ctypes.c_double), ("m_uv", ctypes.c_double),
                ("m_conic", ctypes.c_double), ("m_alpha", ctypes.c_double), ("m_depth", ctypes.c_double),
                ("m_eval", ctypes.c_double), ("m_trel", ctypes.c_double), ("max_leaves", ctypes.c_int64),
                ("lambda_raw", ctypes.c_void_p), ("grad_lambda", ctypes.c_void_p), ("color_rgb", ctypes.c_int64)]


@dataclass
class Settings:
    """Renderer settings.  lambda_opa = 0.35 is the paper's value (Sec. 5.1);
    the rasteriser constants are the 3D Gaussian splatting ones (Sec. 4.4 says
    the pipeline after the slice is that of 3DGS but does not print them)."""

    lambda_opa: float = 0.35
    z_near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)
    jac_guard: float = 1.3
    dilation: float = 0.3
    alpha_max: float = 0.99
    alpha_min: float = 1.0 / 255.0
    t_min: float = 1e-4
    # Float32 error bounds of a renderer working on float32 records; they only
    # feed the decision envelope (render_envelope), never the rendered values.
    # m_uv is in pixels; None: uv_ulps float32 spacings at max(W, H).
    m_uv: float | None = None
    uv_ulps: float = 8.0
    m_conic: float = 6e-5
    m_alpha: float = 3e-5
    m_depth: float = 6e-7
    m_eval: float = 2.4e-7
    m_trel: float = 1.2e-7
    max_leaves: int = 4096
    # False: colour from the degree-3 SH expansion (Sec. 4.2).  True: the No-SH
    # ablation (Sec. 5), rgb = sigmoid(c) with c in the SH degree-0 rows.
    rgb_color: bool = False

    def uv_margin(self, cam) -> float:
        if self.m_uv is not None:
            return float(self.m_uv)
        return float(self.uv_ulps * np.spacing(np.float32(max(int(cam.width), int(cam.height)))))

    def _c(self, cam=None, lambda_raw=None, grad_lambda=None) -> _Set:
        """C settings; lambda_raw / grad_lambda are float64 arrays the caller keeps alive."""
        m_uv = self.uv_margin(cam) if cam is not None else (self.m_uv or 0.0)
        return _Set(self.lambda_opa, self.z_near, (ctypes.c_double * 3)(*self.bg), self.jac_guard,
                    self.dilation, self.alpha_max, self.alpha_min, self.t_min, m_uv, self.m_conic, self.m_alpha,
                    self.m_depth, self.m_eval, self.m_trel, int(self.max_leaves),
                    None if lambda_raw is None else _ptr(lambda_raw),
                    None if grad_lambda is None else _ptr(grad_lambda), int(bool(self.rgb_color)))


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        _lib.orc_preprocess.argtypes = [I64, P, P, P, P]
        _lib.orc_static.argtypes = [I64, P, P]
        _lib.orc_render.argtypes = [I64, P, P, P, I64, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        _lib.orc_render_records.argtypes = [I64, P, P, P, I64, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        _lib.orc_render_records.restype = ctypes.c_int
        _lib.orc_backward.argtypes = [I64, P, P, P, I64, P, P, P, P, ctypes.c_int]
        _lib.orc_slice.argtypes = [I64, P, P, ctypes.c_double, P]
        _lib.orc_sh_basis.argtypes = [I64, P, P]
        _lib.orc_record_vjp.argtypes = [I64, P, P, P, P, P]
        _lib.orc_num_threads.argtypes = [ctypes.c_int]
        _lib.orc_render.restype = ctypes.c_int
        _lib.orc_backward.restype = ctypes.c_int
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _params64(params) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    assert p.ndim == 2 and p.shape[0] == NROWS
    return p


def _cam(cam) -> _Cam:
    c = _Cam()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float64).reshape(9)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float64).reshape(3)]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def num_threads(req: int = 0) -> int:
    return int(lib().orc_num_threads(req))


def _lam(lambda_raw, n):
    """Per-Gaussian raw lambda as a float64 array (or None: the scalar setting)."""
    if lambda_raw is None:
        return None
    a = np.ascontiguousarray(np.asarray(lambda_raw, np.float64).reshape(-1))
    assert a.shape[0] == n
    return a


def preprocess(params, cam, settings: Settings = Settings(), lambda_raw=None) -> dict:
    """Per-Gaussian record for one camera: slice, colour, projection, extents.
    ``lambda_raw`` ([N] or None) gives each Gaussian lambda = sigmoid(raw)."""
    p = _params64(params)
    n = p.shape[1]
    rec = np.zeros((n, NREC), np.float64)
    lam = _lam(lambda_raw, n)
    c, s = _cam(cam), settings._c(cam, lam)
    lib().orc_preprocess(n, _ptr(p), ctypes.byref(c), ctypes.byref(s), _ptr(rec))
    out = {}
    for k, (o, w) in FIELDS.items():
        out[k] = rec[:, o] if w == 1 else rec[:, o:o + w]
    out["alive"] = out["alive"] != 0
    return out


def _render_call(fn, first, cam, settings, pixels, nthreads, lam, envelope):
    """Runs orc_render / orc_render_records (``first`` holds their leading
    arguments) and shapes the outputs."""
    c, s = _cam(cam), settings._c(cam, lam)
    full = pixels is None
    npix = cam.width * cam.height if full else len(pixels)
    pix = None if full else np.ascontiguousarray(np.asarray(pixels, np.int64))
    color = np.zeros((npix, 3), np.float64)
    T = np.zeros(npix, np.float64)
    nc = np.zeros(npix, np.int64)
    if envelope:
        lo = np.zeros((npix, 4), np.float64)
        hi = np.zeros((npix, 4), np.float64)
        impact = np.zeros(npix, np.float64)
        leaves = np.zeros(npix, np.int64)
        flags = np.zeros(npix, np.int32)
        env = [_ptr(lo), _ptr(hi), _ptr(impact), _ptr(leaves), _ptr(flags)]
    else:
        env = [None] * 5
    rc = fn(*first, ctypes.byref(c), ctypes.byref(s), npix, None if full else _ptr(pix), _ptr(color), _ptr(T),
            _ptr(nc), *env, nthreads)
    if rc < 0:
        raise MemoryError("oracle render failed")
    out = {"color": color, "T": T, "ncontrib": nc, "near_z": int(rc)}
    if envelope:
        out.update(lo=lo[:, :3], hi=hi[:, :3], T_lo=lo[:, 3], T_hi=hi[:, 3], leaves=leaves, flags=flags,
                   impact=impact,
                   ambiguous=(flags & (ENV_AMBIGUOUS | ENV_UNRESOLVED)) != 0,
                   kink=(flags & ENV_KINK) != 0, unresolved=(flags & ENV_UNRESOLVED) != 0)
    if full:
        H, W = cam.height, cam.width
        for k, v in list(out.items()):
            if isinstance(v, np.ndarray):
                out[k] = v.T.reshape(v.shape[1], H, W) if v.ndim == 2 else v.reshape(H, W)
    return out


def render(params, cam, settings: Settings = Settings(), pixels=None, nthreads: int = 0, lambda_raw=None):
    """Brute-force render.  Returns (color, T_final, n_contrib, ambiguous); with
    ``pixels=None`` color is [3, H, W] and the others [H, W]; otherwise color is
    [npix, 3] and the others [npix] for the listed row-major pixel ids.
    ``ambiguous`` marks pixels with a threshold decision a float32 renderer may
    take the other way (see ``render_envelope``)."""
    e = render_envelope(params, cam, settings, pixels, nthreads, lambda_raw)
    return e["color"], e["T"], e["ncontrib"], e["ambiguous"]


def render_plain(params, cam, settings: Settings = Settings(), pixels=None, nthreads: int = 0, lambda_raw=None):
    """The brute-force render alone (no decision envelope): (color, T_final, n_contrib)."""
    p = _params64(params)
    e = _render_call(lib().orc_render, (p.shape[1], _ptr(p)), cam, settings, pixels, nthreads,
                     _lam(lambda_raw, p.shape[1]), False)
    return e["color"], e["T"], e["ncontrib"]


def render_envelope(params, cam, settings: Settings = Settings(), pixels=None, nthreads: int = 0,
                    lambda_raw=None) -> dict:
    """Brute-force render plus its decision envelope (test infrastructure).

    ``color``, ``T``, ``ncontrib``: the definition's values.  ``lo`` / ``hi``
    (colour) and ``T_lo`` / ``T_hi``: the range over every combination of
    outcomes of the threshold decisions (alpha >= 1/255, the 1e-4 stop, the
    order at nearly equal depth) that a renderer may legitimately take the
    other way on float32 records, i.e. records within the error bounds
    ``settings.m_*``.  ``leaves``: the number of outcome paths; ``ambiguous``:
    more than one path possible (or the exploration gave up, ``unresolved``);
    ``kink``: a taken Gaussian's alpha is within the error bound of the 0.99
    clamp (the value is continuous there, its derivative is not).
    ``impact``: a bound on the local effect of the undecided decisions (T a
    for a skip, stop or clamp, T a_i a_j for an order); gradient comparisons
    leave out pixels where it is not negligible.
    ``near_z``: Gaussians within the depth margin of z_near, whose culling no
    envelope covers (expected 0).  Shapes as in ``render``."""
    p = _params64(params)
    return _render_call(lib().orc_render, (p.shape[1], _ptr(p)), cam, settings, pixels, nthreads,
                        _lam(lambda_raw, p.shape[1]), True)


RECORD_COLUMNS = ("u", "v", "Qxx", "Qxy", "Qyy", "alpha_cond", "r", "g", "b", "depth", "alive")


def render_records(records, cam, settings: Settings = Settings(), pixels=None, nthreads: int = 0,
                   envelope: bool = True) -> dict:
    """``render_envelope`` from given per-Gaussian records ([m, 11], columns
    RECORD_COLUMNS) instead of parameters."""
    r = np.ascontiguousarray(np.asarray(records, np.float64))
    assert r.ndim == 2 and r.shape[1] == len(RECORD_COLUMNS)
    return _render_call(lib().orc_render_records, (r.shape[0], _ptr(r)), cam, settings, pixels, nthreads, None,
                        envelope)


def records_of(params, cam, settings: Settings = Settings()) -> np.ndarray:
    """The records ``render_records`` takes, computed by ``preprocess``."""
    o = preprocess(params, cam, settings)
    return np.column_stack([o["u"], o["v"], o["conic"], o["alpha_cond"], o["rgb"], o["depth"],
                            o["alive"] | (o["near_cut"] == 1)]).astype(np.float64)


def backward(params, cam, dl_dimage, settings: Settings = Settings(), pixels=None, nthreads: int = 0,
             lambda_raw=None):
    """Analytic gradient of sum(dl_dimage * image) w.r.t. the 76 raw parameter
    rows.  ``dl_dimage`` is [3, H, W] (pixels=None) or [npix, 3].  Returns
    (grad [76, N], g2d [N, 9]) with g2d the per-Gaussian screen-space gradients
    (du, dv, dQxx, dQxy, dQyy, dalpha_cond, dr, dg, db); with ``lambda_raw``
    also the gradient w.r.t. it ([N]) as a third element."""
    p = _params64(params)
    n = p.shape[1]
    lam = _lam(lambda_raw, n)
    glam = None if lam is None else np.zeros(n, np.float64)
    c, s = _cam(cam), settings._c(cam, lam, glam)
    full = pixels is None
    if full:
        npix = cam.width * cam.height
        dl = np.ascontiguousarray(np.asarray(dl_dimage, np.float64).reshape(3, -1).T)
        pix = None
    else:
        npix = len(pixels)
        pix = np.ascontiguousarray(np.asarray(pixels, np.int64))
        dl = np.ascontiguousarray(np.asarray(dl_dimage, np.float64).reshape(npix, 3))
    grad = np.zeros((NROWS, n), np.float64)
    g2d = np.zeros((n, NG2D), np.float64)
    rc = lib().orc_backward(n, _ptr(p), ctypes.byref(c), ctypes.byref(s), npix, None if full else _ptr(pix),
                            _ptr(dl), _ptr(grad), _ptr(g2d), nthreads)
    if rc != 0:
        raise MemoryError("oracle backward failed")
    return (grad, g2d) if lam is None else (grad, g2d, glam)



def static_part(params) -> np.ndarray:
    """The slice's direction-independent part per Gaussian, [22, N]: Sigma_cond
    (xx xy xz yy yz zz), K = Sigma_pd Sigma_d^-1 (row-major), Sigma_d^-1
    (xx xy xz yy yz zz), alpha (Alg. 1 steps 1-3 up to the direction)."""
    p = _params64(params)
    n = p.shape[1]
    out = np.zeros((n, 22), np.float64)
    lib().orc_static(n, _ptr(p), _ptr(out))
    return np.ascontiguousarray(out.T)


def slice_gaussians(params, dirs, lambda_opa: float):
    """Slice every Gaussian at its own unit direction (dirs [N, 3]).  Returns
    (mu_cond [N,3], sigma_cond [N,3,3], D [N], f [N], alpha_cond [N])."""
    p = _params64(params)
    n = p.shape[1]
    d = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(n, 3))
    out = np.zeros((n, 12), np.float64)
    lib().orc_slice(n, _ptr(p), _ptr(d), float(lambda_opa), _ptr(out))
    s = out[:, 3:9]
    sig = np.stack([s[:, [0, 1, 2]], s[:, [1, 3, 4]], s[:, [2, 4, 5]]], axis=1)
    return out[:, 0:3], sig, out[:, 9], out[:, 10], out[:, 11]


def sh_basis(dirs) -> np.ndarray:
    """Real SH basis, degree 3 (16 values) at unit directions [M, 3]."""
    d = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 3))
    out = np.zeros((d.shape[0], 16), np.float64)
    lib().orc_sh_basis(d.shape[0], _ptr(d), _ptr(out))
    return out


def record_vjp(params, cam, g2d, settings: Settings = Settings()) -> np.ndarray:
    """Gradient w.r.t. raw parameters of sum(g2d * (u, v, Q, alpha_cond, rgb))."""
    p = _params64(params)
    n = p.shape[1]
    g = np.ascontiguousarray(np.asarray(g2d, np.float64).reshape(n, NG2D))
    grad = np.zeros((NROWS, n), np.float64)
    c, s = _cam(cam), settings._c(cam)
    lib().orc_record_vjp(n, _ptr(p), ctypes.byref(c), ctypes.byref(s), _ptr(g), _ptr(grad))
    return grad


from .binning import bin_records, tile_grid  # noqa: E402
from .train import adam_step, l1_loss, densify_stats  # noqa: E402
from .density import decompose, decisions, densify  # noqa: E402
from .dssim import l1_dssim_loss, ssim  # noqa: E402

__all__ = ["Settings", "build", "preprocess", "render", "render_plain", "render_envelope", "render_records",
           "records_of", "backward", "slice_gaussians", "sh_basis",
           "record_vjp", "bin_records", "tile_grid", "adam_step", "l1_loss", "densify_stats", "num_threads"]
