"""Whole-frame oracle results computed on a pool of worker processes (test infrastructure).

The arithmetic is that of ``render``, ``voxels``, ``splat`` and ``composite``: this module
only spreads their per-plane and per-view work over processes (planes are independent
given the partition, Alg. 1 "Rasterize" in parallel over chunks; views are independent
given the planes, Alg. 1 steps 6-11) and stores the results as ``.npy`` files.

It forks its workers, so it runs as a program of its own,

    python -m oracle.pool frame --config cluster500k --out DIR [--processes N]

started as a child process by the tests and by the CPU baseline of the benchmark; it never
runs inside a process that has used the GPU.  The frame written to DIR:

    planes.npy   [K,H,W,4] float64 premultiplied planes (Gaussian or filtered voxel planes)
    amb.npy      [K,H,W] bool, texels whose 1/255 inclusion is ambiguous (voxels: none)
    depth.npy    [K] float32 plane depths;  chunk_of.npy, chunk_count.npy  the partition
    views.npy    [V,Ny,Nx,4] float64 (Q_r, Q_g, Q_b, T) of the quilt's views
    vamb.npy     [V,Ny,Nx] bool, pixels that sample an ambiguous texel
    timing.json  wall seconds of the partition, planes and views and the process count
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import composite, geometry, partition, render, splat, voxels

_JOB = {}       # inherited by the forked workers


def default_processes(cap: int = 16) -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def _gaussian_plane(k):
    j = _JOB
    proj = render.chunk_projection(j["scene"], j["cam"], j["geom"], j["part"], k)
    return splat.render_plane(proj, j["geom"].hp, j["geom"].wp)


def _voxel_plane(k):
    j = _JOB
    part = j["part"]
    idx = part.order[part.chunk_start[k]:part.chunk_start[k + 1]]
    return voxels.lowpass(voxels.render_plane(j["scene"], idx, j["cam"], j["geom"])), None


def _view(v):
    j = _JOB
    out, amb = composite.composite(j["planes"], j["depth"], j["cam"], j["geom"], j["dx"], j["dy"], j["interp"],
                                   j["amb"], views=[v])
    return out[0], amb[0]


def _map(fn, n, processes):
    if processes <= 1:
        return [fn(i) for i in range(n)]
    with mp.get_context("fork").Pool(processes) as pool:
        return pool.map(fn, range(n), chunksize=1)


def frame(scene, cam, n_chunk, kind="gaussians", binning="quantile", inv_depth_range=None, dx=None, dy=None,
          interp="nearest", processes=None):
    """Planes of every chunk and the composite of every view (dx, dy float32 offsets)."""
    processes = processes or default_processes()
    t = {"processes": processes}
    g = geometry.derive(cam)
    t0 = time.perf_counter()
    if kind == "voxels":
        part = voxels.partition_voxels(scene, cam, g, n_chunk, binning, inv_depth_range)
    else:
        part = partition.partition(scene["means"], cam, g, n_chunk, binning, inv_depth_range)
    t["partition_s"] = time.perf_counter() - t0
    _JOB.clear()
    _JOB.update(scene=scene, cam=cam, geom=g, part=part)
    t0 = time.perf_counter()
    res = _map(_voxel_plane if kind == "voxels" else _gaussian_plane, n_chunk, processes)
    planes = np.stack([r[0] for r in res])
    amb = np.zeros(planes.shape[:3], bool) if kind == "voxels" else np.stack([r[1] for r in res])
    del res
    t["planes_s"] = time.perf_counter() - t0
    out = dict(planes=planes, amb=amb, depth=part.depth, chunk_of=part.chunk_of, chunk_count=part.chunk_count)
    if dx is not None:
        _JOB.update(planes=planes, depth=part.depth, dx=np.asarray(dx, np.float32), dy=np.asarray(dy, np.float32),
                    interp=interp, amb=None if kind == "voxels" else amb)
        t0 = time.perf_counter()
        res = _map(_view, len(dx), processes)
        out["views"] = np.stack([r[0] for r in res])
        out["vamb"] = np.stack([r[1] for r in res])
        t["views_s"] = time.perf_counter() - t0
    _JOB.clear()
    return out, t


def _main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m oracle.pool")
    ap.add_argument("what", choices=["frame"])
    ap.add_argument("--config", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--processes", type=int, default=0)
    ap.add_argument("--interp", default="nearest")
    ap.add_argument("--no-views", action="store_true")
    a = ap.parse_args(argv)
    import scenegen        # seeded inputs only

    scene, cam, cfg = scenegen.config(a.config)
    kind = "voxels" if cfg["scene"][0] == "voxel" else "gaussians"
    dx = dy = None
    if not a.no_views:
        dx, dy, _, _ = geometry.quilt_views(cam, cfg["vx"], cfg.get("vy", 1))
        dx, dy = dx.astype(np.float32), dy.astype(np.float32)
    res, t = frame(scene, cam, cfg["n_chunk"], kind, cfg["binning"], cfg.get("inv_depth_range"), dx, dy, a.interp,
                   a.processes or None)
    os.makedirs(a.out, exist_ok=True)
    for name, arr in res.items():
        np.save(os.path.join(a.out, name + ".npy"), arr)
    with open(os.path.join(a.out, "timing.json"), "w") as f:
        json.dump(t, f)
    print("oracle frame", a.config, json.dumps(t), flush=True)


if __name__ == "__main__":
    sys.exit(_main())
