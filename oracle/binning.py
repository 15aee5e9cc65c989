"""Integer stage of the rasteriser, as its plain definition (test infrastructure only).

After the slice the method hands its conditional 3D Gaussians to the 3D
Gaussian splatting rasteriser (Sec. 4.4), which bins each projected Gaussian
into the screen tiles its extent overlaps and orders every tile's list by depth.
This module writes that out directly:

* rectangle of tiles: ``tx0 = floor((u - ex) / tile_w)``,
  ``tx1 = floor((u + ex) / tile_w) + 1``, clamped to ``[0, ntx]`` (y alike);
  the subtraction and the multiplication by the exact power of two ``1/tile_w``
  are taken in float32, the precision the GPU takes the same decision in;
* one key per (tile, Gaussian): ``(view_tile_base + ty*ntx + tx) << 32 |
  bits(float32 depth)``, value = entry id ``view*N + gaussian``;
* a stable sort by (key, entry id) (numpy's stable lexsort), and per-tile
  ``[start, end)`` ranges by binary search.
"""
from __future__ import annotations

import numpy as np


def tile_grid(cams, tile_w: int, tile_h: int):
    """Per view (ntx, nty, tile_base) and the total tile count."""
    out, base = [], 0
    for c in cams:
        ntx = -(-int(c.width) // tile_w)
        nty = -(-int(c.height) // tile_h)
        out.append((ntx, nty, base))
        base += ntx * nty
    return out, base


def _rect(center, ext, inv, ntile):
    c = np.asarray(center, np.float32)
    e = np.asarray(ext, np.float32)
    lo = np.floor((c - e) * np.float32(inv)).astype(np.int64)
    hi = np.floor((c + e) * np.float32(inv)).astype(np.int64) + 1
    return np.clip(lo, 0, ntile), np.clip(hi, 0, ntile)


def bin_records(u, v, ex, ey, depth, alive, n: int, cams, tile_w: int, tile_h: int):
    """Bin entries e = view*n + gaussian (all arrays of length n*len(cams)).

    Returns a dict with rect (x0, y0, x1, y1), tiles_touched, keys (uint64,
    sorted), values (int64, sorted) and ranges ([total_tiles, 2])."""
    grid, total = tile_grid(cams, tile_w, tile_h)
    E = n * len(cams)
    alive = np.asarray(alive, bool).reshape(E)
    x0 = np.zeros(E, np.int64); x1 = np.zeros(E, np.int64)
    y0 = np.zeros(E, np.int64); y1 = np.zeros(E, np.int64)
    ntx_e = np.zeros(E, np.int64); base_e = np.zeros(E, np.int64)
    for vi, (ntx, nty, base) in enumerate(grid):
        sl = slice(vi * n, (vi + 1) * n)
        x0[sl], x1[sl] = _rect(np.asarray(u).reshape(E)[sl], np.asarray(ex).reshape(E)[sl], 1.0 / tile_w, ntx)
        y0[sl], y1[sl] = _rect(np.asarray(v).reshape(E)[sl], np.asarray(ey).reshape(E)[sl], 1.0 / tile_h, nty)
        ntx_e[sl] = ntx
        base_e[sl] = base
    tiles = np.where(alive, (x1 - x0) * (y1 - y0), 0)
    ent = np.nonzero(tiles > 0)[0]
    cnt = tiles[ent]
    P = int(cnt.sum())
    rep = np.repeat(ent, cnt)
    # position of each pair inside its entry's rectangle, row-major
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    k = np.arange(P, dtype=np.int64) - first
    w = (x1 - x0)[rep]
    tx = x0[rep] + k % np.maximum(w, 1)
    ty = y0[rep] + k // np.maximum(w, 1)
    tile = base_e[rep] + ty * ntx_e[rep] + tx
    dbits = np.asarray(depth, np.float32).reshape(E).view(np.uint32).astype(np.uint64)
    keys = (tile.astype(np.uint64) << np.uint64(32)) | dbits[rep]
    order = np.lexsort((rep, keys))
    keys, vals = keys[order], rep[order]
    tiles_sorted = (keys >> np.uint64(32)).astype(np.int64)
    t = np.arange(total, dtype=np.int64)
    ranges = np.stack([np.searchsorted(tiles_sorted, t, "left"), np.searchsorted(tiles_sorted, t, "right")], 1)
    return {"rect": np.stack([x0, y0, x1, y1]), "tiles_touched": tiles, "keys": keys, "values": vals,
            "ranges": ranges, "total_tiles": total}
