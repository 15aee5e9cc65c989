"""MI355X (gfx950) renderer for view-conditioned 6D Gaussians.

The hot path -- slice, SH colour, EWA projection, tile binning with an
on-device radix sort, alpha compositing, their backward, the L1 loss and Adam --
is hand-written HIP in ``lib6dgs.so`` behind the C ABI of ``include/sixdgs.h``.
This package is the thin Python layer over it.
"""
from ._lib import Context, SixDGSError, adam, build_cache, default_settings, lib  # noqa: F401
from .render import DEFAULT_LR, Render6D, Renderer, Trainer, render  # noqa: F401
