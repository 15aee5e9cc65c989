"""Host logic of bench.py: the backward's visited (8x8 block, Gaussian) pair
count behind its lane-utilisation figure, against a direct loop over tiles,
blocks and list positions on a small synthetic binning."""
import math

import numpy as np

import bench
from paper_2410_04974_amd import _lib


def _hits(r, x0, y0):
    u, v, qa, qb, qc, al, ex, ey = (float(x) for x in r[:8])
    if not (u + ex >= x0 - 1 and u - ex <= x0 + 8 and v + ey >= y0 - 1 and v - ey <= y0 + 8):
        return False
    lim = 2 * math.log(255 * al) * 1.001 + 1e-3
    xl, yl = x0 - u, y0 - v
    xh, yh = xl + 7, yl + 7
    inx, iny = xl <= 0 <= xh, yl <= 0 <= yh
    if inx and iny:
        return True
    best = math.inf
    if not inx:
        dx = xl if xl > 0 else xh
        dy = min(max(-qb * dx / qc, yl), yh)
        best = min(best, qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy)
    if not iny:
        dy = yl if yl > 0 else yh
        dx = min(max(-qb * dy / qa, xl), xh)
        best = min(best, qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy)
    return best <= lim


def test_visited_block_pairs_matches_a_direct_count():
    rng = np.random.default_rng(1)
    W, H, tw, th = 53, 37, 16, 16  # ragged tiles on both edges
    ntx, nty = -(-W // tw), -(-H // th)
    T, E = ntx * nty, 200
    rec = np.zeros((E, 12), np.float32)
    rec[:, 0] = rng.uniform(-5, W + 5, E)
    rec[:, 1] = rng.uniform(-5, H + 5, E)
    s = rng.uniform(0.5, 6, E)
    rec[:, 2] = 1 / s**2
    rec[:, 3] = rng.uniform(-0.3, 0.3, E) / s**2
    rec[:, 4] = 1 / s**2
    rec[:, 5] = rng.uniform(0.01, 0.99, E)
    rec[:, 6] = rec[:, 7] = 3 * s
    lists = [rng.choice(E, rng.integers(0, 40), replace=False) for _ in range(T)]
    vals = np.concatenate(lists).astype(np.int32)
    starts = np.cumsum([0] + [len(x) for x in lists])
    ranges = np.stack([starts[:-1], starts[1:]], 1).astype(np.int32)
    last = rng.integers(0, 30, W * H).astype(np.int32)

    class Ctx:
        class settings:
            tile_w, tile_h = tw, th

        @staticmethod
        def export(what):
            return {_lib.EXPORT_RECORDS: rec, _lib.EXPORT_VALUES: vals, _lib.EXPORT_RANGES: ranges,
                    _lib.EXPORT_LAST: last}[what]

    class Cam:
        width, height = W, H

    L = last.reshape(H, W)
    want = 0
    for t in range(T):
        tx, ty = t % ntx, t // ntx
        for by in (0, 8):
            for bx in (0, 8):
                ys = range(ty * th + by, min(ty * th + by + 8, H))
                xs = range(tx * tw + bx, min(tx * tw + bx + 8, W))
                wl = max([L[y, x] for y in ys for x in xs], default=0)
                want += sum(1 for j, e in enumerate(lists[t])
                            if j < wl and _hits(rec[e], tx * tw + bx + 0.5, ty * th + by + 0.5))
    assert want > 50
    assert bench.visited_block_pairs(Ctx, Cam) == want
