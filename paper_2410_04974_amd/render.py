"""PyTorch front end: a renderer object holding one library context, the
``Render6D`` autograd function and a fused training step.  PyTorch provides
device memory and the stream; every step of the computation runs in lib6dgs.so.
"""
from __future__ import annotations

import torch

from . import _lib

# Adam learning rates per row group (mu_p, mu_d, Cholesky, SH degree 0,
# SH degrees 1-3, opacity).  1e-2 for the 6D covariance and 1e-3 for the
# direction mean are the paper's (Sec. 5.1); the rest are the 3DGS defaults it
# defers to.
DEFAULT_LR = (1.6e-4, 1e-3, 1e-2, 2.5e-3, 1.25e-4, 5e-2)


class Renderer:
    """Owns a library context (workspace, autotuned settings, the saved state
    of the last forward)."""

    def __init__(self, lambda_opa=0.35, z_near=0.2, bg=(0.0, 0.0, 0.0), tile=(16, 16), batch=0,
                 pair_capacity=0, flags=0, chunk=0, rgb_color=False):
        """rgb_color=True selects the No-SH colour: sigmoid of a per-Gaussian RGB
        held in the SH degree-0 rows (the other SH rows are ignored).  batch /
        chunk 0: the library picks the backward's batch depth and chunk from
        the tile count of each call (``ctx.sizes()`` reports the choice)."""
        if rgb_color:
            flags |= _lib.FLAG_RGB_COLOR
        self.ctx = _lib.Context(lambda_opa=lambda_opa, z_near=z_near, bg=bg, tile_w=tile[0], tile_h=tile[1],
                                batch=batch, pair_capacity=pair_capacity, flags=flags, chunk=chunk)

    def configure(self, **kw):
        if "tile" in kw:
            kw["tile_w"], kw["tile_h"] = kw.pop("tile")
        self.ctx.set_settings(**kw)

    def forward(self, params, cams, out=None, targets=None, dl_dimages=None, loss=None):
        """Images of the cameras; with targets, dl_dimages and loss (a float32
        CUDA [1]) also the L1 loss against the targets and its dL/dI."""
        imgs = out if out is not None else [
            torch.empty((3, c.height, c.width), device=params.device, dtype=torch.float32) for c in cams]
        self.ctx.forward(params, cams, imgs, targets=targets, dl_dimages=dl_dimages, loss=loss)
        return imgs

    def forward_cached(self, params, cache, cams, out=None):
        """Render-only forward from an inference cache (``_lib.build_cache``);
        no backward may follow it."""
        imgs = out if out is not None else [
            torch.empty((3, c.height, c.width), device=params.device, dtype=torch.float32) for c in cams]
        self.ctx.forward_cached(params, cache, cams, imgs)
        return imgs

    def backward(self, params, dl_dimages, grad=None, densify=None):
        g = grad if grad is not None else torch.empty_like(params)
        self.ctx.backward(params, [d.contiguous() for d in dl_dimages], g, densify)
        return g


class Render6D(torch.autograd.Function):
    """images = Render6D.apply(params, renderer, cams); differentiable in params.

    params is a contiguous float32 CUDA tensor [76, N] (layout in include/sixdgs.h).
    Returns one [3, H, W] image per camera.  The renderer keeps the state the
    backward needs, so a renderer serves one forward/backward pair at a time:
    the backward of an output whose renderer has rendered again since raises
    instead of differentiating the later forward (use one renderer per pending
    backward)."""

    @staticmethod
    def forward(ctx, params, renderer, cams):
        params = params.contiguous()
        imgs = renderer.forward(params, cams)
        ctx.renderer = renderer
        ctx.cams = cams
        ctx.generation = renderer.ctx.generation
        ctx.save_for_backward(params)
        return tuple(imgs)

    @staticmethod
    def backward(ctx, *grads):
        if ctx.renderer.ctx.generation != ctx.generation:
            raise RuntimeError("this render's renderer has run another forward since; its backward state is "
                               "gone (use one Renderer per pending backward)")
        (params,) = ctx.saved_tensors
        dl = [g.contiguous() if g is not None else
              torch.zeros((3, c.height, c.width), device=params.device, dtype=torch.float32)
              for g, c in zip(grads, ctx.cams)]
        return ctx.renderer.backward(params, dl), None, None


def render(params, renderer, cams):
    return Render6D.apply(params, renderer, cams)


class Trainer:
    """One training step (render, L1 loss, backward, Adam) entirely in the
    library, on the current stream, with no host synchronisation once the
    renderer has a fixed pair capacity."""

    def __init__(self, params, renderer, lr=DEFAULT_LR, betas=(0.9, 0.999), eps=1e-15, lambda_raw=None,
                 lr_lambda=1e-2, lambda_dssim=0.0):
        """``lambda_raw`` (float32 CUDA [n], or None for the renderer's scalar
        lambda) makes the directional-opacity strength a learnable
        per-Gaussian sigmoid(raw); it is updated by its own Adam while
        ``train_lambda`` is True (the paper trains it over a window of
        iterations and keeps it fixed otherwise).  ``lambda_dssim`` > 0 trains
        with the full 3DGS loss (1 - l) L1 + l (1 - SSIM) (3DGS: l = 0.2);
        0 keeps the plain L1 term."""
        self.params = params
        self.lambda_dssim = lambda_dssim
        self.renderer = renderer
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.grad = torch.empty_like(params)
        self.lr = lr
        self.betas = betas
        self.eps = eps
        self.step_count = 0
        # Adam's step count lives on the device so a captured step advances it on every replay
        self.step_counter = torch.zeros(1, device=params.device, dtype=torch.int32)
        self.loss = torch.zeros(1, device=params.device, dtype=torch.float32)
        self._imgs = None
        self._dl = None
        self.graphs = {}
        self.lambda_raw = lambda_raw
        self.lr_lambda = lr_lambda
        self.train_lambda = lambda_raw is not None
        if lambda_raw is not None:
            self.grad_lambda = torch.zeros_like(lambda_raw)
            self.m_lambda = torch.zeros_like(lambda_raw)
            self.v_lambda = torch.zeros_like(lambda_raw)
            renderer.ctx.set_lambda(lambda_raw, self.grad_lambda)

    def _adam_lambda(self):
        # shares the step's device counter; runs before the parameter Adam advances it
        if self.lambda_raw is not None and self.train_lambda:
            _lib.adam_vec(self.lambda_raw, self.grad_lambda, self.m_lambda, self.v_lambda, self.lr_lambda,
                          step_counter=self.step_counter, beta1=self.betas[0], beta2=self.betas[1], eps=self.eps)

    def step(self, cams, targets, densify=None, fused=True):
        """Render, L1 loss, backward, Adam.  fused=True applies Adam at the end
        of the preprocess backward (the gradient rows stay in LDS and never
        reach memory: 649 against 677 us per step on the 300k-Gaussian
        800x800 step on MI355X); fused=False writes the gradient to self.grad
        and runs the streaming Adam kernel.  Both read and advance the step
        count on the device, so a step can be captured in a graph."""
        if self._imgs is None or [tuple(i.shape) for i in self._imgs] != [(3, c.height, c.width) for c in cams]:
            self._imgs = [torch.empty((3, c.height, c.width), device=self.params.device) for c in cams]
            self._dl = [torch.empty_like(i) for i in self._imgs]
        if self.lambda_dssim > 0:
            self.renderer.forward(self.params, cams, out=self._imgs)
            self.renderer.ctx.l1_dssim_loss(self._imgs, targets, self._dl, self.loss, self.lambda_dssim)
        else:
            # the L1 loss and its gradient formed as the forward writes the pixels
            self.renderer.forward(self.params, cams, out=self._imgs, targets=targets, dl_dimages=self._dl,
                                  loss=self.loss)
        self.step_count += 1
        if fused:
            # a trained lambda shares the step: its Adam runs after this one, then the count moves on
            shared = self.lambda_raw is not None and self.train_lambda
            self.renderer.ctx.backward_adam(self.params, self._dl, self.m, self.v, self.lr, None, self.betas[0],
                                            self.betas[1], self.eps, densify=densify,
                                            step_counter=self.step_counter, advance=not shared)
            if shared:
                self._adam_lambda()
                self.step_counter += 1
        else:
            self.renderer.backward(self.params, self._dl, grad=self.grad, densify=densify)
            self._adam_lambda()
            _lib.adam_devstep(self.params, self.grad, self.m, self.v, self.lr, self.step_counter, self.betas[0],
                              self.betas[1], self.eps)
        return self.loss

    def capture(self, cams, targets, densify=None, warmup=2, key=0):
        """Capture one training step (render, L1, backward, Adam) for these
        cameras as a graph; ``replay(key)`` then runs a step with one launch.
        Several camera sets can be captured under different keys (the camera
        table is part of each capture).  Needs a fixed pair capacity on the
        renderer (no host waits inside a step); warm-up steps are real steps."""
        if self.renderer.ctx.settings.pair_capacity <= 0:
            raise RuntimeError("graph capture needs Renderer(pair_capacity=...) > 0")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step(cams, targets, densify=densify)
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(cams, targets, densify=densify)
        self.step_count -= 1  # capturing did not run a step
        self.graphs[key] = g
        return g

    def replay(self, key=0):
        self.graphs[key].replay()
        self.step_count += 1
        return self.loss

    # -- adaptive density control (Sec. 4.3) -------------------------------------
    def densify(self, stats, extent, grad_threshold=2e-4, percent_dense=0.01, min_opacity=0.01, generator=None):
        """Clone / split / prune from the accumulated statistics ``stats`` ([2, n],
        as filled by ``step(densify=stats)``); the parameters, Adam moments and
        a learnable lambda are replaced by the new set (captured graphs are
        dropped: they refer to the old buffers).  Returns the new count."""
        n = self.params.shape[1]
        noise = torch.randn((2, 3, n), device=self.params.device, generator=generator)
        p, m, v, lam = self.renderer.ctx.densify(self.params, stats, noise, grad_threshold, percent_dense, extent,
                                                 min_opacity, m=self.m, v=self.v, lambda_raw=self.lambda_raw)
        self.params, self.m, self.v = p, m, v
        self.grad = torch.empty_like(p)
        if self.lambda_raw is not None:
            self.lambda_raw = lam
            self.grad_lambda = torch.zeros_like(lam)
            self.m_lambda = torch.zeros_like(lam)
            self.v_lambda = torch.zeros_like(lam)
            self.renderer.ctx.set_lambda(self.lambda_raw, self.grad_lambda)
        self.graphs = {}
        return p.shape[1]

    # -- checkpoint / resume ----------------------------------------------------
    def save(self, path, extra=None):
        """Writes params, Adam moments, the step count and any extra tensors
        (e.g. densification statistics) to an .npz file."""
        import numpy as np
        torch.cuda.synchronize()
        arrays = {"params": self.params.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
                  "step_count": np.array(self.step_count, np.int64),
                  "step_counter": self.step_counter.cpu().numpy()}
        if self.lambda_raw is not None:
            arrays["lambda_raw"] = self.lambda_raw.cpu().numpy()
            arrays["m_lambda"] = self.m_lambda.cpu().numpy()
            arrays["v_lambda"] = self.v_lambda.cpu().numpy()
        for k, t in (extra or {}).items():
            arrays["extra_" + k] = t.cpu().numpy()
        np.savez(path, **arrays)

    def load(self, path):
        """Restores a checkpoint written by save(); returns its extra tensors on the device."""
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            dev = self.params.device
            if tuple(z["params"].shape) != tuple(self.params.shape):
                self.params = torch.empty(tuple(z["params"].shape), device=dev, dtype=torch.float32)
                self.m = torch.empty_like(self.params)
                self.v = torch.empty_like(self.params)
                self.grad = torch.empty_like(self.params)
            self.params.copy_(torch.from_numpy(z["params"]))
            self.m.copy_(torch.from_numpy(z["m"]))
            self.v.copy_(torch.from_numpy(z["v"]))
            self.step_count = int(z["step_count"])
            self.step_counter.copy_(torch.from_numpy(z["step_counter"]))
            if "lambda_raw" in z.files:
                if self.lambda_raw is None or tuple(self.lambda_raw.shape) != tuple(z["lambda_raw"].shape):
                    self.lambda_raw = torch.empty(tuple(z["lambda_raw"].shape), device=dev, dtype=torch.float32)
                    self.grad_lambda = torch.zeros_like(self.lambda_raw)
                    self.m_lambda = torch.zeros_like(self.lambda_raw)
                    self.v_lambda = torch.zeros_like(self.lambda_raw)
                    self.train_lambda = True
                self.lambda_raw.copy_(torch.from_numpy(z["lambda_raw"]))
                self.m_lambda.copy_(torch.from_numpy(z["m_lambda"]))
                self.v_lambda.copy_(torch.from_numpy(z["v_lambda"]))
                self.renderer.ctx.set_lambda(self.lambda_raw, self.grad_lambda)
            extra = {k[len("extra_"):]: torch.from_numpy(z[k]).to(dev) for k in z.files if k.startswith("extra_")}
        self.graphs = {}
        return extra
