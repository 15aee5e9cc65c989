"""ctypes binding of lib6dgs.so: argument marshalling only.

Every computation runs in the HIP library; this module turns torch tensors into
device pointers and the current torch stream into a hipStream_t.  Loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SIXDGS_LIB selects another build of the same library (e.g. to compare two builds)
LIB_PATH = os.environ.get("SIXDGS_LIB", os.path.join(_HERE, "lib6dgs.so"))

OK, ERR_INVALID_ARG, ERR_OOM, ERR_HIP, ERR_CAPACITY, ERR_STATE, ERR_DEBUG = range(7)
MAX_VIEWS = 16
FLAG_COUNTS = 1
FLAG_RGB_COLOR = 2
FLAG_DEBUG = 4
CACHE_ROWS = 22  # rows of the inference cache (SIXDGS_CACHE_ROWS)
EXPORT_RECORDS, EXPORT_TILES, EXPORT_KEYS, EXPORT_VALUES, EXPORT_RANGES, EXPORT_T_FINAL, EXPORT_LAST, \
    EXPORT_COUNTS, EXPORT_SIZES = range(9)
K_PREPROCESS, K_BLEND_FWD, K_BLEND_BWD, K_PREPROCESS_BWD, K_SORT = range(5)
KERNEL_NAMES = {K_PREPROCESS: "preprocess", K_BLEND_FWD: "blend_fwd", K_BLEND_BWD: "blend_bwd",
                K_PREPROCESS_BWD: "preprocess_bwd", K_SORT: "binning"}


class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class Settings(ctypes.Structure):
    _fields_ = [("lambda_opa", ctypes.c_float), ("z_near", ctypes.c_float), ("bg", ctypes.c_float * 3),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("pair_capacity", ctypes.c_int64), ("flags", ctypes.c_int32), ("chunk", ctypes.c_int32)]


class DensitySettings(ctypes.Structure):
    _fields_ = [("grad_threshold", ctypes.c_float), ("percent_dense", ctypes.c_float), ("extent", ctypes.c_float),
                ("min_opacity", ctypes.c_float)]


class BinState(ctypes.Structure):
    """sixdgs_bin_state: host copies of one binning's outputs."""
    _fields_ = [("E", ctypes.c_int64), ("P", ctypes.c_int64), ("T", ctypes.c_int64),
                ("tiles", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("keys", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("ranges", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("chunk", ctypes.c_int32), ("nch", ctypes.c_void_p), ("items", ctypes.c_void_p),
                ("n_items", ctypes.c_int64)]


class SixDGSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lib6dgs status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python __graft_entry__.py build, "
                               "or paper_2410_04974_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        PP = ctypes.POINTER(ctypes.c_void_p)
        L.sixdgs_default_settings.argtypes = [ctypes.POINTER(Settings)]
        L.sixdgs_default_settings.restype = None
        L.sixdgs_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Settings)]
        L.sixdgs_destroy.argtypes = [P]
        L.sixdgs_destroy.restype = None
        L.sixdgs_set_settings.argtypes = [P, ctypes.POINTER(Settings)]
        L.sixdgs_last_error.argtypes = [P]
        L.sixdgs_last_error.restype = ctypes.c_char_p
        L.sixdgs_forward.argtypes = [P, P, I64, ctypes.POINTER(Camera), I32, PP, P]
        L.sixdgs_forward_l1.argtypes = [P, P, I64, ctypes.POINTER(Camera), I32, PP, PP, PP, P, P]
        L.sixdgs_build_cache.argtypes = [P, I64, P, P]
        L.sixdgs_forward_cached.argtypes = [P, P, P, I64, ctypes.POINTER(Camera), I32, PP, P]
        L.sixdgs_backward.argtypes = [P, P, I64, I32, PP, P, P, P]
        L.sixdgs_backward_adam.argtypes = [P, P, I64, I32, PP, P, P, ctypes.POINTER(F), F, F, F, I32, P, P]
        L.sixdgs_backward_adam_devstep.argtypes = [P, P, I64, I32, PP, P, P, ctypes.POINTER(F), F, F, F, P, I32, P,
                                                   P]
        L.sixdgs_l1_loss.argtypes = [P, I32, PP, PP, ctypes.POINTER(I64), PP, P, P]
        L.sixdgs_l1_loss_noalloc.argtypes = [I32, PP, PP, ctypes.POINTER(I64), PP, P, P]
        L.sixdgs_adam.argtypes = [P, P, P, P, I64, ctypes.POINTER(F), F, F, F, I32, P]
        L.sixdgs_adam_devstep.argtypes = [P, P, P, P, I64, ctypes.POINTER(F), F, F, F, P, P]
        L.sixdgs_adam_vec.argtypes = [P, P, P, P, I64, F, F, F, F, I32, P, P]
        L.sixdgs_set_lambda.argtypes = [P, P, P]
        L.sixdgs_l1_dssim_loss.argtypes = [P, I32, PP, PP, ctypes.POINTER(I32), ctypes.POINTER(I32), F, PP, P, P]
        L.sixdgs_decompose.argtypes = [P, I64, P, P, P]
        L.sixdgs_densify_plan.argtypes = [P, P, I64, P, ctypes.POINTER(DensitySettings), ctypes.POINTER(I64), P]
        L.sixdgs_densify_apply.argtypes = [P, P, P, P, P, I64, P, P, P, P, P, I64, P]
        L.sixdgs_bin.argtypes = [P, I64, ctypes.POINTER(Camera), I32, P, P, P, P, P, P, P]
        L.sixdgs_export.argtypes = [P, I32, P, I64, ctypes.POINTER(I64)]
        L.sixdgs_check.argtypes = [P]
        L.sixdgs_debug_check_bins.argtypes = [ctypes.POINTER(BinState), ctypes.c_char_p, I32]
        L.sixdgs_debug_buffer.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(P), ctypes.POINTER(I64)]
        L.sixdgs_set_timing.argtypes = [P, I32]
        L.sixdgs_kernel_time.argtypes = [P, I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]
        for name in ("sixdgs_create", "sixdgs_set_settings", "sixdgs_forward", "sixdgs_forward_l1", "sixdgs_backward",
                     "sixdgs_build_cache", "sixdgs_forward_cached",
                     "sixdgs_backward_adam", "sixdgs_backward_adam_devstep", "sixdgs_l1_loss",
                     "sixdgs_l1_loss_noalloc",
                     "sixdgs_adam", "sixdgs_adam_devstep", "sixdgs_bin", "sixdgs_export", "sixdgs_check",
                     "sixdgs_set_timing", "sixdgs_kernel_time", "sixdgs_debug_check_bins",
                     "sixdgs_debug_buffer"):
            getattr(L, name).restype = I32
        _lib = L
    return _lib


EXPORTED = ["sixdgs_default_settings", "sixdgs_create", "sixdgs_destroy", "sixdgs_set_settings",
            "sixdgs_last_error", "sixdgs_forward", "sixdgs_forward_l1", "sixdgs_build_cache", "sixdgs_forward_cached",
            "sixdgs_backward", "sixdgs_backward_adam", "sixdgs_backward_adam_devstep", "sixdgs_l1_loss",
            "sixdgs_l1_loss_noalloc",
            "sixdgs_l1_dssim_loss",
            "sixdgs_adam", "sixdgs_adam_devstep", "sixdgs_adam_vec", "sixdgs_set_lambda", "sixdgs_decompose",
            "sixdgs_densify_plan", "sixdgs_densify_apply", "sixdgs_bin",
            "sixdgs_export", "sixdgs_check", "sixdgs_set_timing", "sixdgs_kernel_time",
            "sixdgs_debug_check_bins", "sixdgs_debug_buffer"]


def check_bins(tiles, depth, keys, values, ranges, order=None, chunk=0, nch=None, items=None):
    """sixdgs_debug_check_bins on numpy arrays (uint32, except depth float32;
    ranges [T][2], items [n_items][2]).  Returns (status, message)."""
    def arr(a, dt):
        return None if a is None else np.ascontiguousarray(a, dt)
    a = {k: arr(v, np.float32 if k == "depth" else np.uint32)
         for k, v in dict(tiles=tiles, depth=depth, keys=keys, values=values, ranges=ranges, order=order,
                          nch=nch, items=items).items()}
    b = BinState()
    b.E, b.P, b.T = len(a["tiles"]), len(a["keys"]), len(a["ranges"].reshape(-1)) // 2
    for k in ("tiles", "depth", "keys", "values", "ranges", "order", "nch", "items"):
        setattr(b, k, None if a[k] is None else a[k].ctypes.data)
    b.chunk = int(chunk)
    b.n_items = 0 if a["items"] is None else len(a["items"].reshape(-1)) // 2
    msg = ctypes.create_string_buffer(512)
    rc = lib().sixdgs_debug_check_bins(ctypes.byref(b), msg, 512)
    return rc, msg.value.decode()


def default_settings(**kw) -> Settings:
    s = Settings()
    lib().sixdgs_default_settings(ctypes.byref(s))
    for k, v in kw.items():
        if k == "bg":
            s.bg[:] = [float(x) for x in v]
        else:
            setattr(s, k, v)
    return s


def to_camera(cam) -> Camera:
    """Anything with R (3x3), t (3), fx, fy, cx, cy, width, height."""
    c = Camera()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).reshape(9)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32).reshape(3)]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


def _ptrs(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for k, t in enumerate(tensors):
        arr[k] = ctypes.c_void_p(t.data_ptr())
    return arr


def _check_f32_cuda(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")


class Context:
    """One library context: workspace plus the state one forward leaves for its backward."""

    def __init__(self, settings: Settings | None = None, **kw):
        s = settings if settings is not None else default_settings(**kw)
        h = ctypes.c_void_p()
        rc = lib().sixdgs_create(ctypes.byref(h), ctypes.byref(s))
        if rc != OK:
            raise SixDGSError(rc, "create failed (unsupported settings?)")
        self._h = h
        self.settings = s
        # the last forward that left state for a backward: its number (forwards
        # on this context count from 1; 0 = none) and image sizes
        self.generation = 0
        self._fwd_sizes = None

    def close(self):
        if getattr(self, "_h", None):
            lib().sixdgs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rc(self, rc):
        if rc != OK:
            raise SixDGSError(rc, lib().sixdgs_last_error(self._h).decode())

    def set_lambda(self, lambda_raw=None, grad_lambda=None):
        """Learnable per-Gaussian lambda: float32 CUDA tensors [n] (or None), kept
        referenced here while attached."""
        for t, nm in ((lambda_raw, "lambda_raw"), (grad_lambda, "grad_lambda")):
            if t is not None:
                _check_f32_cuda(t, nm)
        self._lambda = (lambda_raw, grad_lambda)
        self._rc(lib().sixdgs_set_lambda(self._h, None if lambda_raw is None else ctypes.c_void_p(lambda_raw.data_ptr()),
                                         None if grad_lambda is None else ctypes.c_void_p(grad_lambda.data_ptr())))

    def densify(self, params, stats, noise, grad_threshold=2e-4, percent_dense=0.01, extent=1.0, min_opacity=0.01,
                m=None, v=None, lambda_raw=None, stream=None):
        """One density-control step (plan, then apply); returns the new params
        and, when given, m, v and lambda_raw, as new tensors."""
        import torch
        _check_f32_cuda(params, "params")
        n = params.shape[1]
        d = DensitySettings(grad_threshold, percent_dense, extent, min_opacity)
        n_out = ctypes.c_int64()
        self._rc(lib().sixdgs_densify_plan(self._h, _vp(params), n, _vp(stats), ctypes.byref(d), ctypes.byref(n_out),
                                           ctypes.c_void_p(_stream(stream))))
        k = n_out.value
        new = lambda: torch.empty((76, k), device=params.device, dtype=torch.float32)
        po = new()
        mo, vo = (new(), new()) if m is not None else (None, None)
        lo = torch.empty(k, device=params.device, dtype=torch.float32) if lambda_raw is not None else None
        self._rc(lib().sixdgs_densify_apply(self._h, _vp(params), _vp(m), _vp(v), _vp(lambda_raw), n, _vp(noise),
                                            _vp(po), _vp(mo), _vp(vo), _vp(lo), k, ctypes.c_void_p(_stream(stream))))
        return po, mo, vo, lo

    def set_settings(self, **kw):
        for k, v in kw.items():
            if k == "bg":
                self.settings.bg[:] = [float(x) for x in v]
            else:
                setattr(self.settings, k, v)
        self._rc(lib().sixdgs_set_settings(self._h, ctypes.byref(self.settings)))

    # -- rendering -------------------------------------------------------------
    def forward(self, params, cams, images, stream=None, targets=None, dl_dimages=None, loss=None):
        """Renders into images; with targets (and dl_dimages, loss) also the L1
        loss and its dL/dI, formed as the pixels are written."""
        n = params.shape[1]
        _check_f32_cuda(params, "params")
        if params.dim() != 2 or params.shape[0] != 76:
            raise ValueError("params must have shape [76, N]")
        if len(images) != len(cams):
            raise ValueError("one image per camera")
        for im, c in zip(images, cams):
            _check_f32_cuda(im, "image")
            if im.numel() != 3 * int(c.width) * int(c.height):
                raise ValueError("each image must hold 3*H*W floats")
        if targets is not None:
            if dl_dimages is None or loss is None or len(targets) != len(cams) or len(dl_dimages) != len(cams):
                raise ValueError("targets, dl_dimages and loss: one target and gradient per camera, and the loss")
            for im, t, g in zip(images, targets, dl_dimages):
                _check_f32_cuda(t, "target")
                _check_f32_cuda(g, "dl_dimage")
                if not (t.numel() == g.numel() == im.numel()):
                    raise ValueError("image, target and gradient sizes differ")
            _check_f32_cuda(loss, "loss")
        ccams = (Camera * len(cams))(*[to_camera(c) for c in cams])
        self._fwd_sizes = None
        if targets is None:
            self._rc(lib().sixdgs_forward(self._h, ctypes.c_void_p(params.data_ptr()), n, ccams, len(cams),
                                          _ptrs(images), ctypes.c_void_p(_stream(stream))))
        else:
            self._rc(lib().sixdgs_forward_l1(self._h, ctypes.c_void_p(params.data_ptr()), n, ccams, len(cams),
                                             _ptrs(images), _ptrs(targets), _ptrs(dl_dimages),
                                             ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(_stream(stream))))
        self.generation += 1
        self._fwd_sizes = [3 * int(c.width) * int(c.height) for c in cams]

    def forward_cached(self, params, cache, cams, images, stream=None):
        """Render-only forward from an inference cache (see build_cache)."""
        n = params.shape[1]
        _check_f32_cuda(params, "params")
        _check_f32_cuda(cache, "cache")
        if params.dim() != 2 or params.shape[0] != 76:
            raise ValueError("params must have shape [76, N]")
        if tuple(cache.shape) != (CACHE_ROWS, n):
            raise ValueError(f"cache must have shape [{CACHE_ROWS}, N]")
        if len(images) != len(cams):
            raise ValueError("one image per camera")
        for im, c in zip(images, cams):
            _check_f32_cuda(im, "image")
            if im.numel() != 3 * int(c.width) * int(c.height):
                raise ValueError("each image must hold 3*H*W floats")
        ccams = (Camera * len(cams))(*[to_camera(c) for c in cams])
        self._fwd_sizes = None  # a render-only forward leaves no state for a backward
        self.generation += 1
        self._rc(lib().sixdgs_forward_cached(self._h, ctypes.c_void_p(params.data_ptr()),
                                             ctypes.c_void_p(cache.data_ptr()), n, ccams, len(cams), _ptrs(images),
                                             ctypes.c_void_p(_stream(stream))))

    def _check_upstream(self, dl_dimages):
        """dL/dI must match the last forward's views one for one (the library
        can check their count, not the sizes of the buffers behind them)."""
        if self._fwd_sizes is None:
            return  # the library reports the missing forward
        if len(dl_dimages) != len(self._fwd_sizes):
            raise ValueError(f"{len(dl_dimages)} dL/dI images for a forward of {len(self._fwd_sizes)} views")
        for k, (t, want) in enumerate(zip(dl_dimages, self._fwd_sizes)):
            _check_f32_cuda(t, "dl_dimage")
            if t.numel() != want:
                raise ValueError(f"dL/dI {k} holds {t.numel()} floats, its view {want}")

    def backward(self, params, dl_dimages, grad, densify=None, stream=None):
        n = params.shape[1]
        for t in dl_dimages:
            _check_f32_cuda(t, "dl_dimage")
        self._check_upstream(dl_dimages)
        _check_f32_cuda(grad, "grad")
        if grad.shape != params.shape:
            raise ValueError("grad must have the shape of params")
        if densify is not None:
            _check_f32_cuda(densify, "densify")
            if densify.numel() != 2 * n:
                raise ValueError("densify must hold [2, N] floats")
        dens = ctypes.c_void_p(densify.data_ptr()) if densify is not None else None
        self._rc(lib().sixdgs_backward(self._h, ctypes.c_void_p(params.data_ptr()), n, len(dl_dimages),
                                       _ptrs(dl_dimages),
                                       ctypes.c_void_p(grad.data_ptr()), dens, ctypes.c_void_p(_stream(stream))))

    def backward_adam(self, params, dl_dimages, m, v, lr, step=None, beta1=0.9, beta2=0.999, eps=1e-15,
                      densify=None, stream=None, step_counter=None, advance=True):
        """Backward fused with the Adam step: the host's step count (from 1),
        or step_counter (int32 CUDA [1]: step = counter + 1, advanced by the
        kernel when ``advance``)."""
        n = params.shape[1]
        for t in dl_dimages:
            _check_f32_cuda(t, "dl_dimage")
        self._check_upstream(dl_dimages)
        for t, nm in ((m, "m"), (v, "v")):
            _check_f32_cuda(t, nm)
            if t.shape != params.shape:
                raise ValueError(f"{nm} must have the shape of params")
        if densify is not None:
            _check_f32_cuda(densify, "densify")
            if densify.numel() != 2 * n:
                raise ValueError("densify must hold [2, N] floats")
        lrs = (ctypes.c_float * 6)(*[float(x) for x in lr])
        dens = ctypes.c_void_p(densify.data_ptr()) if densify is not None else None
        head = (self._h, ctypes.c_void_p(params.data_ptr()), n, len(dl_dimages), _ptrs(dl_dimages),
                ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), lrs, beta1, beta2, eps)
        if step_counter is not None:
            import torch
            if not (step_counter.is_cuda and step_counter.dtype == torch.int32 and step_counter.numel() >= 1):
                raise ValueError("step_counter must be an int32 CUDA tensor")
            self._rc(lib().sixdgs_backward_adam_devstep(*head, ctypes.c_void_p(step_counter.data_ptr()),
                                                        int(bool(advance)), dens, ctypes.c_void_p(_stream(stream))))
        else:
            self._rc(lib().sixdgs_backward_adam(*head, int(step), dens, ctypes.c_void_p(_stream(stream))))
        self._fwd_sizes = None  # the parameters moved: the forward's state is spent
        self.generation += 1

    def l1_loss(self, images, targets, dl_dimages, loss, stream=None):
        for a, b, g in zip(images, targets, dl_dimages):
            for t in (a, b, g):
                _check_f32_cuda(t, "image")
            if not (a.numel() == b.numel() == g.numel()):
                raise ValueError("image, target and gradient sizes differ")
        _check_f32_cuda(loss, "loss")
        numel = (ctypes.c_int64 * len(images))(*[t.numel() for t in images])
        self._rc(lib().sixdgs_l1_loss(self._h, len(images), _ptrs(images), _ptrs(targets), numel,
                                      _ptrs(dl_dimages), ctypes.c_void_p(loss.data_ptr()),
                                      ctypes.c_void_p(_stream(stream))))

    def l1_dssim_loss(self, images, targets, dl_dimages, loss, lambda_dssim=0.2, stream=None):
        """(1 - lambda) L1 + lambda (1 - SSIM) over [3, H, W] views, dL/dI into dl_dimages."""
        for a, b, g in zip(images, targets, dl_dimages):
            for t in (a, b, g):
                _check_f32_cuda(t, "image")
            if not (a.dim() == 3 and a.shape[0] == 3 and a.shape == b.shape == g.shape):
                raise ValueError("images, targets and gradients must share one [3, H, W] shape per view")
        _check_f32_cuda(loss, "loss")
        hs = (ctypes.c_int32 * len(images))(*[t.shape[1] for t in images])
        ws = (ctypes.c_int32 * len(images))(*[t.shape[2] for t in images])
        self._rc(lib().sixdgs_l1_dssim_loss(self._h, len(images), _ptrs(images), _ptrs(targets), hs, ws,
                                            float(lambda_dssim), _ptrs(dl_dimages), ctypes.c_void_p(loss.data_ptr()),
                                            ctypes.c_void_p(_stream(stream))))

    def bin(self, n, cams, u, v, ex, ey, depth, alive, stream=None):
        import torch
        for t in (u, v, ex, ey, depth):
            _check_f32_cuda(t, "record array")
            if t.numel() != n * len(cams):
                raise ValueError("record arrays must hold n * ncam entries")
        if not (alive.is_cuda and alive.dtype == torch.int32 and alive.numel() == n * len(cams)):
            raise ValueError("alive must be an int32 CUDA tensor of n * ncam entries")
        ccams = (Camera * len(cams))(*[to_camera(c) for c in cams])
        self._fwd_sizes = None  # the binning replaces the forward's state
        self.generation += 1
        self._rc(lib().sixdgs_bin(self._h, n, ccams, len(cams), *[ctypes.c_void_p(t.data_ptr()) for t in
                                                                   (u, v, ex, ey, depth, alive)],
                                  ctypes.c_void_p(_stream(stream))))

    def check(self):
        self._rc(lib().sixdgs_check(self._h))

    # -- read-back (synchronous) ----------------------------------------------------
    def sizes(self):
        out = np.zeros(7, np.int64)
        w = ctypes.c_int64()
        self._rc(lib().sixdgs_export(self._h, EXPORT_SIZES, out.ctypes.data_as(ctypes.c_void_p), 56, ctypes.byref(w)))
        return {"entries": int(out[0]), "pairs": int(out[1]), "tiles": int(out[2]), "binned": int(out[3]),
                "pixels": int(out[4]), "batch": int(out[5]), "chunk": int(out[6])}

    def export(self, what):
        sz = self.sizes()
        E, P, T, X = sz["entries"], sz["pairs"], sz["tiles"], sz["pixels"]
        spec = {EXPORT_RECORDS: (np.float32, (E, 12)), EXPORT_TILES: (np.int32, (E,)),
                EXPORT_KEYS: (np.uint64, (P,)), EXPORT_VALUES: (np.int32, (P,)),
                EXPORT_RANGES: (np.int32, (T, 2)), EXPORT_T_FINAL: (np.float32, (X,)),
                EXPORT_LAST: (np.int32, (X,)), EXPORT_COUNTS: (np.int32, (X,))}
        dt, shape = spec[what]
        out = np.zeros(shape, dt)
        w = ctypes.c_int64()
        self._rc(lib().sixdgs_export(self._h, what, out.ctypes.data_as(ctypes.c_void_p), out.nbytes,
                                     ctypes.byref(w)))
        return out

    # -- timing ----------------------------------------------------------------------
    def set_timing(self, mask):
        self._rc(lib().sixdgs_set_timing(self._h, int(mask)))

    def kernel_time(self, kernel):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._rc(lib().sixdgs_kernel_time(self._h, kernel, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def decompose(params, stream=None):
    """Rotation R [3, 3, N] and scale S [3, N] of every Gaussian's conditional covariance."""
    import torch
    _check_f32_cuda(params, "params")
    n = params.shape[1]
    R = torch.empty((3, 3, n), device=params.device, dtype=torch.float32)
    S = torch.empty((3, n), device=params.device, dtype=torch.float32)
    rc = lib().sixdgs_decompose(_vp(params), n, _vp(R), _vp(S), ctypes.c_void_p(_stream(stream)))
    if rc != OK:
        raise SixDGSError(rc, "decompose failed")
    return R, S


def adam_vec(p, grad, m, v, lr, step=1, step_counter=None, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    """Adam on one float32 CUDA vector with one learning rate; with a device
    step counter the step is counter + 1 and the counter is left as it is."""
    import torch
    for t, nm in ((p, "p"), (grad, "grad"), (m, "m"), (v, "v")):
        _check_f32_cuda(t, nm)
        if t.shape != p.shape:
            raise ValueError("p, grad, m and v must share one shape")
    if step_counter is not None and not (step_counter.is_cuda and step_counter.dtype == torch.int32
                                         and step_counter.numel() == 1):
        raise ValueError("step_counter must be a one-element int32 CUDA tensor")
    rc = lib().sixdgs_adam_vec(ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                               ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), p.numel(), float(lr),
                               beta1, beta2, eps, int(step),
                               None if step_counter is None else ctypes.c_void_p(step_counter.data_ptr()),
                               ctypes.c_void_p(_stream(stream)))
    if rc != OK:
        raise SixDGSError(rc, "adam_vec failed (bad arguments)")


def build_cache(params, out=None, stream=None):
    """Inference cache of params [76, N]: a [22, N] float32 CUDA tensor holding
    Sigma_cond, K = Sigma_pd Sigma_d^-1, Sigma_d^-1 and alpha per Gaussian."""
    import torch
    _check_f32_cuda(params, "params")
    n = params.shape[1]
    cache = out if out is not None else torch.empty((CACHE_ROWS, n), device=params.device, dtype=torch.float32)
    _check_f32_cuda(cache, "cache")
    if tuple(cache.shape) != (CACHE_ROWS, n):
        raise ValueError(f"cache must have shape [{CACHE_ROWS}, N]")
    rc = lib().sixdgs_build_cache(ctypes.c_void_p(params.data_ptr()), n, ctypes.c_void_p(cache.data_ptr()),
                                  ctypes.c_void_p(_stream(stream)))
    if rc != OK:
        raise SixDGSError(rc, "build_cache failed (bad arguments)")
    return cache


def l1_loss_noalloc(images, targets, dl_dimages, loss, stream=None):
    """sixdgs_l1_loss_noalloc: the L1 loss and its gradient with the library's
    fixed per-device scratch (no context, no allocation)."""
    for a, b, g in zip(images, targets, dl_dimages):
        for t in (a, b, g):
            _check_f32_cuda(t, "image")
        if not (a.numel() == b.numel() == g.numel()):
            raise ValueError("image, target and gradient sizes differ")
    if not (len(images) == len(targets) == len(dl_dimages)):
        raise ValueError("one target and one gradient per image")
    _check_f32_cuda(loss, "loss")
    numel = (ctypes.c_int64 * len(images))(*[t.numel() for t in images])
    rc = lib().sixdgs_l1_loss_noalloc(len(images), _ptrs(images), _ptrs(targets), numel, _ptrs(dl_dimages),
                                      ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(_stream(stream)))
    if rc != OK:
        raise SixDGSError(rc, "l1_loss_noalloc failed (bad arguments, or the scratch lookup failed)")


def adam_devstep(params, grad, m, v, lr, step_counter, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    """Adam with the step count in a device int32 tensor (capturable in a graph)."""
    import torch
    for t, nm in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _check_f32_cuda(t, nm)
        if t.shape != params.shape:
            raise ValueError("params, grad, m and v must share one shape")
    if not (step_counter.is_cuda and step_counter.dtype == torch.int32 and step_counter.numel() == 1):
        raise ValueError("step_counter must be a one-element int32 CUDA tensor")
    lrs = (ctypes.c_float * 6)(*[float(x) for x in lr])
    rc = lib().sixdgs_adam_devstep(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                   ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), params.shape[1],
                                   lrs, beta1, beta2, eps, ctypes.c_void_p(step_counter.data_ptr()),
                                   ctypes.c_void_p(_stream(stream)))
    if rc != OK:
        raise SixDGSError(rc, "adam failed (bad arguments)")


def adam(params, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    """One fused Adam step over [76, N] in place."""
    for t, nm in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _check_f32_cuda(t, nm)
        if t.shape != params.shape:
            raise ValueError("params, grad, m and v must share one shape")
    lrs = (ctypes.c_float * 6)(*[float(x) for x in lr])
    rc = lib().sixdgs_adam(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                           ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), params.shape[1], lrs,
                           beta1, beta2, eps, int(step), ctypes.c_void_p(_stream(stream)))
    if rc != OK:
        raise SixDGSError(rc, "adam failed (bad arguments)")
