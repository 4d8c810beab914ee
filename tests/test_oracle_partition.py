"""Pins of the oracle's keys, cull and chunking (Alg. 1 CulledDepth / FindQuantile /
Sort_and_Chunk, Sec. 4.4): brute force with Python's own sort, integer identities, and
native float32 arithmetic for the float32 decision programs."""
import ctypes
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

import scenegen
from oracle import decisions, geometry, partition

HERE = os.path.dirname(__file__)


@pytest.fixture(scope="module")
def fp32lib():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "fp32_ref.so")
    subprocess.check_call(["gcc", "-O0", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                           os.path.join(HERE, "fp32_ref.c"), "-o", so, "-lm"])
    return ctypes.CDLL(so)


def _ptr(a, t=ctypes.c_float):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _scene_with_edge_cases(n, seed):
    s = scenegen.small_scene(n, seed, xy=2.5, z=(-0.5, 8.0))
    m = s["means"]
    m[::17, 2] = m[::13, 2][: m[::17].shape[0]]      # duplicate keys
    m[5, 2] = -0.0
    m[6] = [np.nan, 0.0, 3.0]
    m[7] = [0.0, 0.0, np.inf]
    m[8, 2] = m[9, 2]
    return s


@pytest.mark.parametrize("rot", [False, True])
def test_keys_and_cull_match_native_float32(fp32lib, rot):
    rng = np.random.default_rng(7)
    R = np.eye(3)
    if rot:
        q = rng.normal(size=4)
        from oracle.project import quat_to_rot
        R = quat_to_rot(q[None])[0]
    cam = scenegen.camera(200, 150, 55.0, 2.5, math.radians(30.0), R=R, t=(0.1, -0.2, 0.3))
    g = geometry.derive(cam)
    c = decisions.constants(g, cam)
    s = _scene_with_edge_cases(4000, 11)
    key, vis = decisions.keys_and_cull(s["means"], cam, c)
    n = s["means"].shape[0]
    kref = np.zeros(n, np.float32)
    vref = np.zeros(n, np.int32)
    Rf = np.asarray(cam.R, np.float32)
    tf = np.asarray(cam.t, np.float32)
    fp32lib.keys_cull(n, _ptr(s["means"]), _ptr(Rf), _ptr(tf), ctypes.c_float(c.d_forward),
                      ctypes.c_float(c.z_near), ctypes.c_float(c.guard_x), ctypes.c_float(c.guard_y),
                      _ptr(kref), _ptr(vref, ctypes.c_int))
    fin = np.isfinite(kref)
    assert np.array_equal(key.view(np.uint32)[fin], kref.view(np.uint32)[fin])
    assert np.array_equal(vis, vref.astype(bool))
    assert 0 < vis.sum() < n


def test_plane_coefficients_match_native_float32(fp32lib):
    cam, cfg = scenegen.config_camera("cluster500k")
    g = geometry.derive(cam)
    c = decisions.constants(g, cam)
    dx, dy, _, _ = geometry.quilt_views(cam, 45, 1)
    dx32 = dx.astype(np.float32)
    d = np.sort(np.random.default_rng(1).uniform(g.d_forward + 0.2, 20.0, 64)).astype(np.float32)
    pc = decisions.plane_coeffs32(c, d, dx32, dy.astype(np.float32))
    b = np.zeros(64, np.float32)
    C = np.zeros((64, 45), np.float32)
    Cn = np.zeros((64, 45), np.float32)
    fp32lib.plane_coeffs(64, _ptr(d), 45, _ptr(dx32), ctypes.c_float(c.d_forward), ctypes.c_float(c.inv_focal),
                         ctypes.c_float(c.ratio_x), ctypes.c_float(c.fpx), ctypes.c_float(c.cpx),
                         _ptr(b), _ptr(C), _ptr(Cn))
    assert np.array_equal(pc.bx.view(np.uint32), b.view(np.uint32))
    assert np.array_equal(pc.Cx.view(np.uint32), C.view(np.uint32))
    assert np.array_equal(pc.Cxn.view(np.uint32), Cn.view(np.uint32))
    xs = np.arange(g.nx).astype(np.float32)
    for k, v in ((0, 0), (31, 22), (63, 44)):
        X, _ = decisions.texel_coords32(pc, c, k, v, np.arange(g.nx), np.arange(g.ny), nearest=True)
        Xr = np.zeros(g.nx, np.float32)
        fp32lib.texel_coords(g.nx, _ptr(xs), ctypes.c_float(c.cx), ctypes.c_float(pc.bx[k]),
                             ctypes.c_float(pc.Cxn[k, v]), _ptr(Xr))
        assert np.array_equal(X.view(np.uint32), Xr.view(np.uint32))


def _brute_order(key, vis):
    items = sorted((float(key[i]), i) for i in range(key.size) if vis[i])
    return np.array([i for _, i in items], dtype=np.int64)


@pytest.mark.parametrize("K", [1, 3, 16, 64])
def test_quantile_against_brute_force(K):
    cam = scenegen.camera(160, 160, 50.0, 2.0, math.radians(40.0))
    g = geometry.derive(cam)
    s = _scene_with_edge_cases(3000, K)
    p = partition.partition(s["means"], cam, g, K, "quantile")
    order = _brute_order(p.key, p.visible)
    assert np.array_equal(p.order, order)
    nv = order.size
    # chunk of rank r is the number of chunks whose share of ranks has started: floor(r K / N_vis)
    for r in range(nv):
        assert p.chunk_of[order[r]] == (r * K) // nv
    assert np.all(p.chunk_of[~p.visible] == -1)
    cnt = np.bincount(p.chunk_of[p.visible], minlength=K)
    assert np.array_equal(cnt, p.chunk_count) and cnt.max() - cnt.min() <= 1 and cnt.sum() == nv
    ks = sorted(float(p.key[i]) for i in order)
    pos = 0
    for k in range(K):
        members = ks[pos:pos + cnt[k]]
        pos += cnt[k]
        assert p.depth[k] == np.float32(members[(len(members) - 1) // 2])   # lower median
        assert members[0] <= p.depth[k] <= members[-1]


def test_quantile_degenerate_cases():
    cam = scenegen.camera(64, 64, 50.0, 2.0, math.radians(40.0))
    g = geometry.derive(cam)
    s = scenegen.small_scene(5, 3)
    p = partition.partition(s["means"], cam, g, 8, "quantile")      # fewer primitives than chunks
    nv = p.order.size
    assert nv == 5 and p.chunk_count.sum() == 5 and np.all(p.chunk_count <= 1)
    for k in range(1, 8):
        if p.chunk_count[k] == 0:
            assert p.depth[k] == p.depth[k - 1]
    s["means"][:, 2] = -5.0                                         # nothing visible
    p = partition.partition(s["means"], cam, g, 4, "quantile")
    assert p.order.size == 0 and np.all(p.chunk_count == 0) and np.all(p.depth == np.float32(cam.d_focal))


def test_inverse_depth_bins():
    cam, cfg = scenegen.config_camera("uniform10k")
    g = geometry.derive(cam)
    s = scenegen.uniform_scene(3000, seed=9)
    s["means"][:40, 2] = np.linspace(1.0, 7.0, 40)                  # keys outside [2, 6] clamp
    K = cfg["n_chunk"]
    lo, hi = cfg["inv_depth_range"]
    p = partition.partition(s["means"], cam, g, K, "inv_depth", (lo, hi))
    E = decisions.inv_depth_edges32(K, lo, hi)
    assert np.all(np.diff(E) > 0) and E[0] > lo and E[-1] < hi
    for i in range(0, s["means"].shape[0], 7):
        if p.visible[i]:
            assert p.chunk_of[i] == sum(1 for e in E if e <= p.key[i])
    assert np.array_equal(p.order, _brute_order(p.key, p.visible))
    # d_k is the harmonic midpoint of the float64 edges E_k, E_{k+1}
    Ef = [lo] + [1.0 / (1.0 / lo + (i / K) * (1.0 / hi - 1.0 / lo)) for i in range(1, K)] + [hi]
    for k in range(K):
        assert p.depth[k] == pytest.approx(2.0 / (1.0 / Ef[k] + 1.0 / Ef[k + 1]), rel=1e-7)
    assert np.all(np.diff(p.chunk_sorted) >= 0)
