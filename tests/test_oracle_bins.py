"""Pins of the tile-list oracle (Sec. 4.4, Alg. 1 "Rasterize"): the must set covers every
texel the splat includes (brute force), must is inside may, and the list checker accepts
lists made from the must set in (key, index) order while rejecting a missing entry, an
entry out of order, an entry of another chunk, a duplicate and an entry beyond may."""
import math

import numpy as np
import pytest

import scenegen
from oracle import bins, geometry, partition, project, render, splat


def _setup(n=400, seed=3, res=70, K=4):
    scene = scenegen.small_scene(n, seed)
    cam = scenegen.camera(res, res - 9, 50.0, 3.0, math.radians(30.0))
    g = geometry.derive(cam)
    part = partition.partition(scene["means"], cam, g, K)
    return scene, cam, g, part, K


def test_must_covers_every_included_texel():
    scene, cam, g, part, K = _setup()
    must, may = bins.tile_lists(scene, cam, g, part, tile=16)
    n_all = scene["means"].shape[0]
    tiles_x = (g.wp + 15) // 16
    got = set(must.tolist())
    checked = 0
    for k in range(K):
        idx = part.order[part.chunk_start[k]:part.chunk_start[k + 1]]
        pr = project.project_reference(scene, idx, cam, g)
        ys, xs = np.meshgrid(np.arange(g.hp), np.arange(g.wp), indexing="ij")
        for r, i in enumerate(idx):
            d = np.stack([xs - pr.mean2d[r, 0], ys - pr.mean2d[r, 1]], -1)
            q = np.einsum("...i,ij,...j->...", d, pr.conic[r], d)
            inc = math.log(pr.opacity[r]) - 0.5 * q >= splat.LN_ALPHA_MIN
            for ty, tx in set(zip((ys[inc] // 16).tolist(), (xs[inc] // 16).tolist())):
                assert ((ty * tiles_x + tx) * K + k) * n_all + i in got
                checked += 1
    assert checked > 500
    assert np.isin(must, may).all() and may.size >= must.size


def _lists_from(codes, part, n_buckets):
    n_all = part.chunk_of.shape[0]
    b, i = codes // n_all, codes % n_all
    rk = bins.ranks(part)[i]
    o = np.lexsort((rk, b))
    b, i = b[o], i[o]
    starts = np.searchsorted(b, np.arange(n_buckets + 1))
    return starts, i


@pytest.mark.parametrize("tile", [8, 16])
def test_checker_accepts_must_lists_and_rejects_mistakes(tile):
    scene, cam, g, part, K = _setup(seed=5)
    must, may = bins.tile_lists(scene, cam, g, part, tile=tile)
    nb = ((g.wp + tile - 1) // tile) * ((g.hp + tile - 1) // tile) * K
    starts, ent = _lists_from(must, part, nb)
    stats = bins.check_lists(starts, ent, must, may, part, nb, K)
    assert stats["beyond_must"] == 0 and stats["entries"] == must.size
    starts2, ent2 = _lists_from(may, part, nb)                     # the widest allowed lists pass too
    bins.check_lists(starts2, ent2, must, may, part, nb, K)
    long = int(np.argmax(np.diff(starts)))
    s0 = starts[long]
    assert starts[long + 1] - s0 >= 2
    bad = ent.copy()
    bad[s0], bad[s0 + 1] = bad[s0 + 1], bad[s0]                     # out of order
    with pytest.raises(AssertionError):
        bins.check_lists(starts, bad, must, may, part, nb, K)
    with pytest.raises(AssertionError):                             # a missing entry
        st = starts.copy()
        st[long + 1:] -= 1
        bins.check_lists(st, np.delete(ent, s0), must, may, part, nb, K)
    other = np.nonzero((part.chunk_of >= 0) & (part.chunk_of != long % K))[0][0]
    bad = ent.copy()
    bad[s0] = other                                                 # another chunk's Gaussian
    with pytest.raises(AssertionError):
        bins.check_lists(starts, bad, must, may, part, nb, K)
    with pytest.raises(AssertionError):                             # a duplicate
        st = starts.copy()
        st[long + 1:] += 1
        bins.check_lists(st, np.insert(ent, s0, ent[s0]), must, may, part, nb, K)
    far = [b for b in range(nb) if b % K == long % K and abs(b // K - long // K) > 3]
    with pytest.raises(AssertionError):                             # an entry far outside its box
        st, en = starts.copy(), ent.copy()
        b = far[0]
        pos = st[b]
        en = np.insert(en, pos, ent[s0])
        st[b + 1:] += 1
        bins.check_lists(st, en, must, may, part, nb, K)
