"""Batched rendering (lf_batch_*): several scenes of different sizes, plane counts, view
counts, dtypes and field kinds rendered by one call, on per-scene streams or phase by phase
over the (scene, item) work list, optionally captured into one HIP graph and autotuned.
Every output must equal, bit for bit, the same scene rendered alone with lf_build_mpi +
lf_composite (whose parity with the oracle the other GPU tests establish), on every graph
replay."""
import math

import numpy as np
import pytest
import torch

import scenegen
from oracle import geometry
from paper_2508_18540_amd import torch_api as T
from tests.gpu_util import announce, ctx

pytestmark = pytest.mark.gpu

# (Gaussians, resolution, N_chunk, views (vx, vy), binning, plane dtype, interp); the last
# scene is a 2D quilt (three vertical offsets) with UNORM8 planes
SCENES = [
    (20_000, 128, 16, (5, 1), "quantile", torch.float32, "nearest"),
    (40_000, 192, 32, (9, 1), "inv_depth", torch.float16, "bilinear"),
    (60_000, 256, 64, (16, 1), "quantile", torch.bfloat16, "nearest"),
    (30_000, 160, 8, (24, 1), "quantile", torch.float16, "nearest"),
    (25_000, 144, 12, (4, 3), "quantile", torch.uint8, "nearest"),
    (35_000, 160, 16, (5, 1), "quantile", torch.float32, "nearest"),
]


def _scenes():
    out = []
    for i, (n, res, K, (vx, vy), binning, pdt, interp) in enumerate(SCENES):
        cam = scenegen.camera(res, res, 50.0, 2.0, math.radians(40.0), math.radians(12.0) if vy > 1 else 0.0)
        dx, dy, _, _ = geometry.quilt_views(cam, vx, vy)
        out.append(dict(scene=T.to_device(scenegen.cluster_scene(n, seed=40 + i)), cam=cam, n_chunk=K,
                        views=T.views_of(dx.astype(np.float32), dy.astype(np.float32)), binning=binning,
                        inv_depth_range=(1.0, 20.0) if binning == "inv_depth" else None, plane_dtype=pdt,
                        interp=interp))
    # a voxel field (its splat is not one of the work list's)
    cam = scenegen.camera(96, 96, 50.0, 4.0, math.radians(40.0))
    vox = scenegen.voxel_scene(res=32, n_occupied=2000, seed=6)
    vox["density"] = (vox["density"] * np.float32(0.1)).astype(np.float32)
    dx, dy, _, _ = geometry.quilt_views(cam, 7, 1)
    out.append(dict(scene=T.to_device(vox), cam=cam, n_chunk=8, views=T.views_of(dx.astype(np.float32), dy.astype(np.float32)),
                    binning="quantile", inv_depth_range=None, plane_dtype=torch.float16, interp="nearest"))
    return out


def _eager(sc):
    o = T.build_mpi(ctx(), sc["scene"], sc["cam"], sc["n_chunk"], sc["binning"], sc["inv_depth_range"],
                    dtype=sc["plane_dtype"])
    img = T.composite(ctx(), o["rgba"], o["depth"], sc["cam"], sc["views"], sc["interp"])
    torch.cuda.synchronize()
    return o["rgba"].clone(), o["depth"].clone(), img.clone()


def _same(b, refs):
    torch.cuda.synchronize()
    for i, (o, (rgba, depth, img)) in enumerate(zip(b.outs, refs)):
        assert torch.equal(o["depth"], depth), i
        assert torch.equal(o["rgba"], rgba), i
        assert torch.equal(o["views"], img), i


@pytest.mark.parametrize("graph,worklist", [(False, False), (True, False), (False, True), (True, True)])
def test_batch_matches_single_scene_calls(graph, worklist):
    announce("batch", "graph" if graph else "eager", "work list" if worklist else "streams")
    scs = _scenes()
    refs = [_eager(sc) for sc in scs]
    b = T.Batch(ctx(), scs, graph=graph, worklist=worklist)
    for rep in range(3):
        for o in b.outs:                                   # eager work between runs / replays
            o["views"].zero_()
            o["rgba"].fill_(7.0)
        torch.cuda.synchronize()
        b.run()
        _same(b, refs)
        x = torch.randn(1 << 20, device="cuda")
        float((x * x).sum())                               # unrelated eager kernels and a sync
    b.close()


@pytest.mark.parametrize("worklist", [False, True])
def test_batch_autotuned_groups(worklist):
    """The autotuned view groups and row tiles (64-pixel waves or 256-pixel row tiles) give
    the same results as the defaults; a second batch of the same shapes takes the cached
    choices."""
    announce("batch autotune", "work list" if worklist else "streams")
    scs = _scenes()
    refs = [_eager(sc) for sc in scs]
    b = T.Batch(ctx(), scs, graph=True, autotune=True, worklist=worklist)
    gs, ts = b.groups(), b.tiles()
    print("autotuned view groups", gs, "row tiles", ts)
    assert all(g in (4, 8, 12, 16) for g in gs) and all(t in (64, 256) for t in ts)
    b.run()
    _same(b, refs)
    b.close()
    again = T.Batch(ctx(), scs, graph=True, autotune=True, worklist=worklist)
    assert again.groups() == gs and again.tiles() == ts
    again.close()


def test_composite_row_tiles_match_wave_tiles(monkeypatch):
    """The 256-pixel row-tile form of the composite (LF_COMPOSITE_TILE=256, the row kernel
    over every segment) equals the default one-wave form bit for bit."""
    announce("composite row tiles")
    for sc in _scenes()[:3]:
        rgba, depth, img = _eager(sc)
        monkeypatch.setenv("LF_COMPOSITE_TILE", "256")
        alt = T.composite(ctx(), rgba, depth, sc["cam"], sc["views"], sc["interp"])
        torch.cuda.synchronize()
        monkeypatch.delenv("LF_COMPOSITE_TILE")
        assert torch.equal(alt, img)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_stats_reports_each_scene(graph):
    """lf_batch_stats after a run: every scene's counters, and a scene whose build overflows
    its tile-list capacity (large footprints, the default capacity of 65536 entries, no
    probe) named in the LF_ERR_CAPACITY it returns, the other scenes unaffected."""
    from paper_2508_18540_amd import _lib as L
    announce("batch stats", "graph" if graph else "streams")
    scenes = _scenes()[:2]
    cam = scenegen.camera(256, 256, 50.0, 2.0, math.radians(40.0))
    dx, dy, _, _ = geometry.quilt_views(cam, 5, 1)
    big = scenegen.small_scene(1500, 7, xy=1.0, z=(2.5, 4.0), log_scale=(-0.6, 0.2))
    scenes.insert(1, dict(scene=T.to_device(big), cam=cam, n_chunk=8, probe=False,
                          views=T.views_of(dx.astype(np.float32), dy.astype(np.float32))))
    b = T.Batch(ctx(), scenes, graph=graph)
    b.run()
    info, n_failed, st = b.stats(check=False)
    assert st == L.LF_ERR_CAPACITY and n_failed == 1, (st, n_failed)
    assert [i.overflow for i in info] == [0, 1, 0]
    assert info[1].entries_needed > info[1].entry_capacity
    for i in (0, 2):
        assert 0 < info[i].entries_needed <= info[i].entry_capacity and info[i].stalled == 0
        assert info[i].n_visible > 0
    with pytest.raises(L.LFError, match="scene 1"):
        b.stats()
    b.close()
    ok = T.Batch(ctx(), _scenes()[:2], graph=graph)
    ok.run()
    info, n_failed, st = ok.stats()
    assert st == L.LF_OK and n_failed == 0 and len(info) == 2
    ok.close()
