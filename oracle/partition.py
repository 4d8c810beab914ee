"""Depth sorting and chunking (Alg. 1: CulledDepth, FindQuantile, Sort_and_Chunk; Sec. 4.4).

Primitives inside the reference frustum are sorted by their base-camera depth
key (ties by primitive index) and split into N_chunk chunks.  Two rules:

* quantile (Sec. 4.4): chunks hold nearly equal numbers of primitives, chunk of
  rank r is floor(r * K / N_vis); the plane depth d_k is the lower median key of
  the chunk (rank lo_k + floor((n_k - 1)/2)); an empty chunk is a transparent plane
  at the previous plane's depth (at D_focal if no primitive is visible);
* inverse depth: K planes uniform in 1/z over [z_lo, z_hi]; the chunk of a key is
  the number of interior edges E_i <= key (keys outside the range clamp into the
  end chunks); d_k is the edge formula evaluated at i = k + 1/2.

Each primitive belongs to exactly one chunk, chosen by its centre depth (Sec. 4.4).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import decisions


@dataclass
class Partition:
    key: np.ndarray           # [N] float32 depth keys
    visible: np.ndarray       # [N] bool
    order: np.ndarray         # [N_vis] primitive indices sorted by (key, index)
    chunk_sorted: np.ndarray  # [N_vis] chunk of each rank
    chunk_of: np.ndarray      # [N] chunk per primitive, -1 if culled
    chunk_count: np.ndarray   # [K]
    chunk_start: np.ndarray   # [K+1] first rank of each chunk
    depth: np.ndarray         # [K] float32 plane depths d_k


def sort_visible(key: np.ndarray, visible: np.ndarray) -> np.ndarray:
    idx = np.nonzero(visible)[0]
    return idx[np.lexsort((idx, key[idx].astype(np.float64)))]


def quantile(key, visible, n_chunk: int, d_focal: float) -> Partition:
    order = sort_visible(key, visible)
    nv = order.size
    ranks = np.arange(nv, dtype=np.int64)
    chunk_sorted = (ranks * n_chunk) // max(nv, 1)
    start = np.array([(k * nv + n_chunk - 1) // n_chunk for k in range(n_chunk + 1)], dtype=np.int64)
    count = np.diff(start)
    depth = np.empty(n_chunk, dtype=np.float32)
    prev = np.float32(d_focal)
    ks = key[order]
    for k in range(n_chunk):
        if count[k] > 0:
            prev = ks[start[k] + (count[k] - 1) // 2]
        depth[k] = prev
    return _finish(key, visible, order, chunk_sorted, start, count, depth, n_chunk)


def inverse_depth(key, visible, n_chunk: int, z_lo: float, z_hi: float) -> Partition:
    order = sort_visible(key, visible)
    edges = decisions.inv_depth_edges32(n_chunk, z_lo, z_hi)
    chunk_sorted = np.searchsorted(edges, key[order], side="right").astype(np.int64)
    count = np.bincount(chunk_sorted, minlength=n_chunk).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(count)]).astype(np.int64)
    k = np.arange(n_chunk, dtype=np.float64)
    depth = (1.0 / (1.0 / z_lo + ((k + 0.5) / n_chunk) * (1.0 / z_hi - 1.0 / z_lo))).astype(np.float32)
    return _finish(key, visible, order, chunk_sorted, start, count, depth, n_chunk)


def _finish(key, visible, order, chunk_sorted, start, count, depth, n_chunk):
    chunk_of = np.full(key.shape[0], -1, dtype=np.int32)
    chunk_of[order] = chunk_sorted.astype(np.int32)
    return Partition(key=key, visible=visible, order=order, chunk_sorted=chunk_sorted,
                     chunk_of=chunk_of, chunk_count=count.astype(np.int32), chunk_start=start,
                     depth=depth)


def partition(points32, cam, geom, n_chunk: int, binning: str = "quantile", inv_depth_range=None) -> Partition:
    """Keys, cull and chunking for a primitive set with centres ``points32`` [N,3] float32."""
    c = decisions.constants(geom, cam)
    key, vis = decisions.keys_and_cull(points32, cam, c)
    if binning == "quantile":
        return quantile(key, vis, n_chunk, geom.d_focal)
    if binning == "inv_depth":
        lo, hi = inv_depth_range
        return inverse_depth(key, vis, n_chunk, lo, hi)
    raise ValueError(binning)
