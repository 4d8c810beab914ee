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
                 (with ``--no-save`` the only file: the benchmark's CPU baseline)

``--target`` renders the workload's perturbed copy instead (the gradient workload's target
views).  ``python -m oracle.pool batch --index i --out DIR`` writes, for scene i of the
batched workload, its partition and the oracle's values at seeded sample texels and view
pixels (``texels.npz``, ``pixels.npz``: positions, values, ambiguity flags).
``python -m oracle.pool fd --config grad200k --out DIR`` renders the perturbed target views
(``target.npy``) and the planes of the scene, then takes footprint-local central differences
of the frozen-decision L2 loss (``grad.footprint_fd``) for seeded (Gaussian, parameter) pairs
in parallel and writes them to ``fd.npz`` (see ``fd_pairs``).  ``bins`` writes the bounds of
the (tile, chunk) lists of a Gaussian workload (``bins.chunk_lists`` per chunk): ``must.npy``
and ``may.npy``.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import bins, composite, geometry, grad, partition, project, render, splat, voxels

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


def _bins_job(k):
    j = _JOB
    return bins.chunk_lists(j["scene"], j["cam"], j["geom"], j["part"], k)


def _fd_job(c):
    j = _JOB
    key, i, jj = j["cands"][c]
    return grad.footprint_fd(j["scene"], j["cam"], j["part"], j["planes"], j["dx"], j["dy"], j["target"], i, key, jj,
                             j["steps"][key])


FD_STEPS = {"means": 1e-4, "log_scales": 1e-4, "quats": 1e-4, "opacity": 1e-5, "rgb": 1e-3}


def fd_pairs(scene, cam, cfg, n_pairs=64, n_draws=48, seed=17, processes=None):
    """Central differences of the gradient workload's loss on seeded pairs.

    Two halves of n_pairs/2 (Gaussian, parameter) pairs, each the first non-ambiguous pairs
    with support among n_draws seeded draws (key uniform over the five parameter tensors,
    component uniform): the uniform half draws the Gaussian uniformly from the visible ones;
    the front half from the visible Gaussians that the planes in front of theirs do not hide,
    i.e. whose reference-ray transmittance through the planes in front, at the texel of the
    projected mean, is at least 1/4 (most Gaussians of a dense scene are hidden, and their
    differences vanish), and whose support fits 49 x 49 texels (a footprint that large
    already reaches 45 views x ~2500 pixels; larger ones cost more and meet more Gaussians
    at a threshold)."""
    processes = processes or default_processes()
    K = cfg["n_chunk"]
    dx, dy, _, _ = geometry.quilt_views(cam, cfg["vx"], 1)
    dx, dy = dx.astype(np.float32), dy.astype(np.float32)
    tgt, _ = frame(scenegen_target(scene, cfg), cam, K, dx=dx, dy=dy, processes=processes)
    target = tgt["views"].astype(np.float32).astype(np.float64)        # float32, as a GPU loss reads it
    del tgt
    base, _ = frame(scene, cam, K, processes=processes)
    g = geometry.derive(cam)
    part = partition.partition(scene["means"], cam, g, K)
    vis = np.nonzero(part.chunk_of >= 0)[0]
    # the planes are parametrised by the reference camera, so texel t of every plane lies on
    # one reference ray: T in front of plane k at t is the product of (1 - A) of planes < k
    t_front = np.cumprod(np.concatenate([np.ones((1, g.hp, g.wp)), 1.0 - base["planes"][:-1, ..., 3]]), axis=0)
    pr = project.project_reference(scene, vis, cam, g)
    mx = np.clip(np.floor(pr.mean2d[:, 0] + 0.5), 0, g.wp - 1).astype(np.int64)
    my = np.clip(np.floor(pr.mean2d[:, 1] + 0.5), 0, g.hp - 1).astype(np.int64)
    inside = (pr.mean2d[:, 0] >= -0.5) & (pr.mean2d[:, 0] < g.wp - 0.5) & (pr.mean2d[:, 1] >= -0.5) & \
        (pr.mean2d[:, 1] < g.hp - 0.5)
    hx, hy, sup = splat.support_halfwidth(pr, np.zeros(vis.size))
    compact = sup & (hx <= 24.0) & (hy <= 24.0)
    front = vis[inside & compact & (t_front[part.chunk_of[vis], my, mx] >= 0.25)]
    del t_front
    rng = np.random.default_rng(seed)
    cands = []
    for pool_ in (vis, front):
        for _ in range(n_draws):
            key = grad.KEYS[rng.integers(0, 5)]
            i = int(rng.choice(pool_))
            jj = int(rng.integers(0, scene[key].shape[1])) if scene[key].ndim == 2 else None
            cands.append((key, i, jj))
    _JOB.clear()
    _JOB.update(scene=scene, cam=cam, part=part, planes=base["planes"], dx=dx, dy=dy, target=target, cands=cands,
                steps=FD_STEPS)
    res = _map(_fd_job, len(cands), processes)
    _JOB.clear()
    half = n_pairs // 2
    pick = []
    for h0 in (0, n_draws):
        ok = [c for c in range(h0, h0 + n_draws) if res[c][2] and not res[c][1]]
        pick += ok[:half]
    return dict(key=np.array([grad.KEYS.index(cands[c][0]) for c in pick]), index=np.array([cands[c][1] for c in pick]),
                comp=np.array([-1 if cands[c][2] is None else cands[c][2] for c in pick]),
                fd=np.array([res[c][0] for c in pick]), uniform=np.array([c < n_draws for c in pick]),
                n_candidates=len(cands), n_front=len(front), n_visible=len(vis),
                n_ambiguous=sum(1 for r in res if r[2] and r[1]), n_no_support=sum(1 for r in res if not r[2])), target


def scenegen_target(scene, cfg):
    import scenegen
    return scenegen.perturbed_target(scene, cfg["target_seed"])


def _main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m oracle.pool")
    ap.add_argument("what", choices=["frame", "batch", "fd", "bins"])
    ap.add_argument("--draws", type=int, default=48)
    ap.add_argument("--config")
    ap.add_argument("--index", type=int, default=0)
    ap.add_argument("--target", action="store_true")
    ap.add_argument("--planes", type=int, default=2)
    ap.add_argument("--texels", type=int, default=300)
    ap.add_argument("--pixels", type=int, default=200)
    ap.add_argument("--out", required=True)
    ap.add_argument("--processes", type=int, default=0)
    ap.add_argument("--interp", default="nearest")
    ap.add_argument("--no-views", action="store_true")
    ap.add_argument("--no-save", action="store_true", help="frame: time only, write timing.json alone")
    a = ap.parse_args(argv)
    import scenegen        # seeded inputs only

    if a.what == "batch":
        return _batch_main(a)
    scene, cam, cfg = scenegen.config(a.config)
    if a.what == "bins":
        t0 = time.perf_counter()
        g = geometry.derive(cam)
        part = partition.partition(scene["means"], cam, g, cfg["n_chunk"], cfg["binning"], cfg.get("inv_depth_range"))
        _JOB.clear()
        _JOB.update(scene=scene, cam=cam, geom=g, part=part)
        res = _map(_bins_job, cfg["n_chunk"], a.processes or default_processes())
        _JOB.clear()
        os.makedirs(a.out, exist_ok=True)
        np.save(os.path.join(a.out, "must.npy"), np.sort(np.concatenate([m for m, _ in res])))
        np.save(os.path.join(a.out, "may.npy"), np.sort(np.concatenate([m for _, m in res])))
        print("oracle bins", a.config, "%.1f s" % (time.perf_counter() - t0), flush=True)
        return 0
    if a.what == "fd":
        t0 = time.perf_counter()
        pairs, target = fd_pairs(scene, cam, cfg, n_draws=a.draws, processes=a.processes or None)
        os.makedirs(a.out, exist_ok=True)
        np.save(os.path.join(a.out, "target.npy"), target)
        np.savez(os.path.join(a.out, "fd.npz"), **pairs)
        print("oracle fd", a.config, "pairs", len(pairs["fd"]), "candidates", pairs["n_candidates"], "visible",
              pairs["n_visible"], "unhidden", pairs["n_front"], "ambiguous",
              pairs["n_ambiguous"], "without support", pairs["n_no_support"], "%.1f s" % (time.perf_counter() - t0),
              flush=True)
        return 0
    if a.target:
        scene = scenegen.perturbed_target(scene, cfg["target_seed"])
    kind = "voxels" if cfg["scene"][0] == "voxel" else "gaussians"
    dx = dy = None
    if not a.no_views:
        dx, dy, _, _ = geometry.quilt_views(cam, cfg["vx"], cfg.get("vy", 1))
        dx, dy = dx.astype(np.float32), dy.astype(np.float32)
    res, t = frame(scene, cam, cfg["n_chunk"], kind, cfg["binning"], cfg.get("inv_depth_range"), dx, dy, a.interp,
                   a.processes or None)
    os.makedirs(a.out, exist_ok=True)
    for name, arr in ({} if a.no_save else res).items():
        np.save(os.path.join(a.out, name + ".npy"), arr)
    with open(os.path.join(a.out, "timing.json"), "w") as f:
        json.dump(t, f)
    print("oracle frame", a.config, json.dumps(t), flush=True)


def batch_samples(scene, cam, n_chunk, n_views, n_planes, n_texels, n_pixels, seed=0):
    """Partition of one batch scene and the oracle at seeded samples: n_texels texels of each
    of n_planes random planes, and n_pixels pixels of the quilt's views (nearest)."""
    g = geometry.derive(cam)
    part = partition.partition(scene["means"], cam, g, n_chunk)
    rng = np.random.default_rng(seed)
    cache = {}

    def texel_fn(k, iy, ix):
        if k not in cache:
            cache[k] = render.chunk_projection(scene, cam, g, part, k)
        return splat.blend_texels(cache[k], ix, iy)

    tk, ty, tx, tv, ta = [], [], [], [], []
    for k in rng.choice(n_chunk, n_planes, replace=False):
        iy, ix = rng.integers(0, g.hp, n_texels), rng.integers(0, g.wp, n_texels)
        v, am = texel_fn(int(k), iy, ix)
        tk.append(np.full(n_texels, k)), ty.append(iy), tx.append(ix), tv.append(v), ta.append(am)
    dx, dy, _, _ = geometry.quilt_views(cam, n_views, 1)
    dx, dy = dx.astype(np.float32), dy.astype(np.float32)
    pix = np.stack([rng.integers(0, n_views, n_pixels), rng.integers(0, cam.ny, n_pixels),
                    rng.integers(0, cam.nx, n_pixels)], 1)
    pv, pa = composite.composite_at(texel_fn, part.depth, cam, g, dx, dy, "nearest", pix)
    return dict(chunk_of=part.chunk_of, chunk_count=part.chunk_count, depth=part.depth,
                texels=dict(k=np.concatenate(tk), y=np.concatenate(ty), x=np.concatenate(tx), value=np.concatenate(tv),
                            ambiguous=np.concatenate(ta)),
                pixels=dict(pix=pix, value=pv, ambiguous=pa))


def _batch_main(a):
    import scenegen

    t0 = time.perf_counter()
    scene, cam, K, V = scenegen.batch_scene(a.index)
    res = batch_samples(scene, cam, K, V, a.planes, a.texels, a.pixels, seed=a.index)
    os.makedirs(a.out, exist_ok=True)
    for name in ("chunk_of", "chunk_count", "depth"):
        np.save(os.path.join(a.out, name + ".npy"), res[name])
    np.savez(os.path.join(a.out, "texels.npz"), **res["texels"])
    np.savez(os.path.join(a.out, "pixels.npz"), **res["pixels"])
    print("oracle batch scene", a.index, "%.1f s" % (time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    sys.exit(_main())
