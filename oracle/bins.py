"""The (tile, chunk) lists of the splat, float64 (Sec. 4.4, Alg. 1 "Rasterize"; test
infrastructure).

Alg. 1 rasterises every chunk with a tile-based rasteriser: the plane is cut into square
tiles and each tile keeps, per chunk, the list of the chunk's Gaussians that can cover one
of its texels, in the chunk's front-to-back (depth key, index) order.  Membership is
decided from the Gaussian's support S = {p : o G(p) >= 1/255} (Sec. 4.4 inherits the 1/255
cut of 3D Gaussian splatting):

* a Gaussian MUST be listed in every tile its support's bounding box over texel centres,
  [ceil(mx - hx), floor(mx + hx)] x [ceil(my - hy), floor(my + hy)] with the exact
  half-widths hx = sqrt(2 ln(255 o) Sigma'_xx), hy likewise, meets (a list that is a
  superset of the support is what the splat needs; the box is the tightest such rectangle);
* it MAY be listed in the tiles of that box widened by a relative 3e-3 and 3e-3 texel (a
  float32 kernel widens its box by a small margin so rounding never drops a texel).

``tile_lists`` returns, per chunk, the must and may sets as sorted codes
bucket * N + gaussian with bucket = tile * K + chunk and tile = ty * tiles_x + tx, plus the
rank of every Gaussian in the (key, index) order, which orders each list.
"""
from __future__ import annotations

import math

import numpy as np

from . import render, splat

MAY_REL = 3e-3
MAY_ABS = 3e-3


def _box_tiles(mx, my, hx, hy, wp, hp, tile):
    x0, x1 = max(0, math.ceil(mx - hx)), min(wp - 1, math.floor(mx + hx))
    y0, y1 = max(0, math.ceil(my - hy)), min(hp - 1, math.floor(my + hy))
    if x0 > x1 or y0 > y1:
        return None
    return x0 // tile, x1 // tile, y0 // tile, y1 // tile


def chunk_lists(scene, cam, geom, part, k: int, tile: int = 16):
    """(must, may) codes of chunk k's Gaussians, each an int64 array of bucket * N + index."""
    idx = part.order[part.chunk_start[k]:part.chunk_start[k + 1]]
    n_all = part.chunk_of.shape[0]
    K = len(part.depth)
    tiles_x = (geom.wp + tile - 1) // tile
    must, may = [], []
    if idx.size == 0:
        z = np.zeros(0, np.int64)
        return z, z
    proj = render.chunk_projection(scene, cam, geom, part, k)
    hx, hy, ok = splat.support_halfwidth(proj, np.zeros(idx.size))
    for r, i in enumerate(idx):
        if not ok[r]:
            continue
        mx, my = proj.mean2d[r]
        for h_x, h_y, out in ((hx[r], hy[r], must), (hx[r] * (1 + MAY_REL) + MAY_ABS, hy[r] * (1 + MAY_REL) + MAY_ABS, may)):
            t = _box_tiles(mx, my, h_x, h_y, geom.wp, geom.hp, tile)
            if t is None:
                continue
            tx0, tx1, ty0, ty1 = t
            ty, tx = np.meshgrid(np.arange(ty0, ty1 + 1), np.arange(tx0, tx1 + 1), indexing="ij")
            bucket = (ty.reshape(-1) * tiles_x + tx.reshape(-1)) * K + k
            out.append(bucket.astype(np.int64) * n_all + int(i))
    cat = lambda a: np.sort(np.concatenate(a)) if a else np.zeros(0, np.int64)  # noqa: E731
    return cat(must), cat(may)


def ranks(part) -> np.ndarray:
    """Position of every visible Gaussian in the (key, index) order (-1 if culled)."""
    r = np.full(part.chunk_of.shape[0], -1, np.int64)
    r[part.order] = np.arange(part.order.size)
    return r


def tile_lists(scene, cam, geom, part, tile: int = 16, chunks=None):
    """must, may: sorted int64 codes over the selected chunks (all by default)."""
    K = len(part.depth)
    res = [chunk_lists(scene, cam, geom, part, k, tile) for k in (range(K) if chunks is None else chunks)]
    return np.sort(np.concatenate([m for m, _ in res])), np.sort(np.concatenate([m for _, m in res]))


def check_lists(bucket_start, entries, must, may, part, n_buckets: int, K: int):
    """Compare GPU lists with the oracle's bounds.  Returns a dict of counts; raises
    AssertionError on a list that misses a must entry, holds an entry outside may, holds a
    Gaussian of another chunk, or is out of (key, index) order."""
    n_all = part.chunk_of.shape[0]
    bucket_start = np.asarray(bucket_start, np.int64)
    entries = np.asarray(entries, np.int64)
    assert bucket_start.shape[0] == n_buckets + 1 and bucket_start[-1] == entries.shape[0]
    counts = np.diff(bucket_start)
    assert (counts >= 0).all()
    bucket_of = np.repeat(np.arange(n_buckets, dtype=np.int64), counts)
    assert np.array_equal(part.chunk_of[entries], bucket_of % K), "an entry sits in another chunk's list"
    rk = ranks(part)[entries]
    same = bucket_of[1:] == bucket_of[:-1]
    assert (rk[1:][same] > rk[:-1][same]).all(), "a list is not in (key, index) order"
    got = np.sort(bucket_of * n_all + entries)
    assert np.unique(got).size == got.size, "a Gaussian listed twice in one list"
    missing = np.setdiff1d(must, got, assume_unique=True)
    extra = np.setdiff1d(got, may, assume_unique=True)
    assert missing.size == 0, f"{missing.size} required entries missing, e.g. bucket {missing[0] // n_all} " \
                              f"Gaussian {missing[0] % n_all}"
    assert extra.size == 0, f"{extra.size} entries beyond the support's widened box, e.g. bucket {extra[0] // n_all} " \
                            f"Gaussian {extra[0] % n_all}"
    return dict(entries=int(got.size), must=int(must.size), may=int(may.size),
                beyond_must=int(np.setdiff1d(got, must, assume_unique=True).size))
