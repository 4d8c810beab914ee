"""Pins of the oracle's swizzle blending (Sec. 4.3, Eqs. 6-7, Alg. 1): the zero-baseline
identity with the conventional per-view render, an opaque front plane, monotone
transmittance, exact translation of nearest views, mirror symmetry, and plain loops."""
import math

import numpy as np
import pytest

import scenegen
from oracle import composite, decisions, geometry, render


@pytest.mark.parametrize("K", [1, 2, 5])
def test_zero_baseline_equals_per_view_render(K):
    """phi = 0, P_s = 1: the reference camera is the base camera and every view is the base
    view, so compositing depth-contiguous chunks with the over operator reproduces a single
    front-to-back render of all Gaussians, for any number of chunks."""
    cam = scenegen.camera(48, 40, 50.0, 2.0, 0.0)
    sc = scenegen.small_scene(60, 5)
    mpi = render.build_mpi_gaussians(sc, cam, K)
    g = mpi.geom
    out, amb = composite.composite(mpi.planes, mpi.depth, cam, g, np.zeros(3, np.float32),
                                   np.zeros(3, np.float32), "nearest", mpi.ambiguous)
    ref, _ = render.render_view(sc, cam, 0.0, 0.0, visible=mpi.part.visible)
    for v in range(3):
        assert np.allclose(out[v, ..., :3], ref[..., :3], atol=1e-12)
        assert np.allclose(out[v, ..., 3], 1.0 - ref[..., 3], atol=1e-12)
    assert ref[..., 3].max() > 0.5


def _planes(K, H, W, seed, **kw):
    return scenegen.random_planes(K, H, W, seed, **kw)


CAM = scenegen.camera(40, 32, 50.0, 2.0, math.radians(30.0))
G = geometry.derive(CAM)
DX, DY, _, _ = geometry.quilt_views(CAM, 5, 1)
DX32, DY32 = DX.astype(np.float32), DY.astype(np.float32)


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_opaque_front_plane_hides_the_rest(interp):
    p = _planes(4, G.hp, G.wp, 1, depth_range=(G.d_forward + 0.5, 6.0))
    rgba = p["rgba"].astype(np.float64)
    rgba[0, ..., 3] = 1.0
    only = rgba[:1].copy()
    out, _ = composite.composite(rgba, p["depth"], CAM, G, DX32, DY32, interp)
    ref, _ = composite.composite(only, p["depth"][:1], CAM, G, DX32, DY32, interp)
    # wherever the front sample lies inside the plane the pixel is fully covered by it
    covered = ref[..., 3] < 1e-15
    assert covered.mean() > 0.5
    assert np.allclose(out[covered], ref[covered], atol=1e-15)


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_transmittance_monotone_and_bounded(interp):
    p = _planes(6, G.hp, G.wp, 2, depth_range=(G.d_forward + 0.5, 9.0))
    prev = None
    for K in range(1, 7):
        out, _ = composite.composite(p["rgba"][:K], p["depth"][:K], CAM, G, DX32, DY32, interp)
        T = out[..., 3]
        assert np.all(T >= 0) and np.all(T <= 1) and np.all(out[..., :3] >= 0)
        assert np.all(out[..., :3] <= (1 - T)[..., None] + 1e-12)     # colour bounded by coverage
        if prev is not None:
            assert np.all(T <= prev + 1e-15)
        prev = T


def test_nearest_views_are_translations():
    """Planes at one depth with b = 1 and offsets that differ by whole texels: each view is
    the previous view shifted by that many texels (zeros shifted in)."""
    cam = scenegen.camera(40, 24, 50.0, 2.0, 0.0)        # D_forward = 0 => slope exactly 1
    g = geometry.derive(cam)
    c = decisions.constants(g, cam)
    d = np.float32(4.0)
    gx = c.fpx * ((np.float32(1.0) - d * c.inv_focal) / (d - c.d_forward))
    steps = np.array([0, 1, 3, -2], dtype=np.float32)
    dx = (steps / gx).astype(np.float32)
    pc = decisions.plane_coeffs32(c, np.array([d] * 3, np.float32), dx, np.zeros(4, np.float32))
    shift = pc.Cxn[0] - pc.Cxn[0, 0]
    assert pc.bx[0] == 1.0 and np.array_equal(shift, np.round(shift))   # precondition: whole texels
    p = _planes(3, g.hp, g.wp, 3)
    out, _ = composite.composite(p["rgba"], np.array([d] * 3, np.float32), cam, g, dx,
                                 np.zeros(4, np.float32), "nearest")
    for v in range(1, 4):
        s = int(shift[v])
        ref = np.zeros_like(out[0])
        ref[..., 3] = 1.0
        if s >= 0:
            ref[:, :g.nx - s] = out[0][:, s:]
        else:
            ref[:, -s:] = out[0][:, :g.nx + s]
        # columns whose source left the plane are transparent in both
        assert np.allclose(out[v], ref, atol=1e-15), v


def test_mirror_symmetry_bilinear():
    """Mirroring the planes left-right and the view offsets maps view v onto the mirror of
    the view with the opposite offset (bilinear sampling is continuous, so float32
    coordinate rounding only perturbs at the 1e-5 level)."""
    cam = scenegen.camera(40, 40, 50.0, 2.0, math.radians(30.0))
    g = geometry.derive(cam)
    dx, _, _, _ = geometry.quilt_views(cam, 5, 1)
    dx32 = dx.astype(np.float32)
    assert np.array_equal(dx32, -dx32[::-1])
    p = _planes(5, g.hp, g.wp, 4, depth_range=(g.d_forward + 0.5, 8.0))
    out, _ = composite.composite(p["rgba"], p["depth"], cam, g, dx32, np.zeros(5, np.float32), "bilinear")
    mir, _ = composite.composite(p["rgba"][:, :, ::-1], p["depth"], cam, g, dx32, np.zeros(5, np.float32), "bilinear")
    for v in range(5):
        assert np.allclose(out[v], mir[4 - v][:, ::-1], atol=1e-4)


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_plain_loops(interp):
    """Alg. 1 written as scalar loops over pixels, planes and taps."""
    p = _planes(3, G.hp, G.wp, 6, depth_range=(G.d_forward + 0.3, 5.0))
    out, _ = composite.composite(p["rgba"], p["depth"], CAM, G, DX32, DY32, interp)
    c = decisions.constants(G, CAM)
    pc = decisions.plane_coeffs32(c, p["depth"], DX32, DY32)
    P = p["rgba"].astype(np.float64)
    for v in (0, 2, 4):
        for y in range(0, G.ny, 3):
            for x in range(0, G.nx, 2):
                Q = np.zeros(3)
                T = 1.0
                for k in range(3):
                    X, Y = decisions.texel_coords32(pc, c, k, v, [x], [y], interp == "nearest")
                    X, Y = float(X[0]), float(Y[0])
                    if interp == "nearest":
                        taps = [(math.floor(Y), math.floor(X), 1.0)]
                    else:
                        x0, y0 = math.floor(X), math.floor(Y)
                        fx, fy = X - x0, Y - y0
                        taps = [(y0, x0, (1 - fx) * (1 - fy)), (y0, x0 + 1, fx * (1 - fy)),
                                (y0 + 1, x0, (1 - fx) * fy), (y0 + 1, x0 + 1, fx * fy)]
                    s = np.zeros(4)
                    for iy, ix, w in taps:
                        if 0 <= iy < G.hp and 0 <= ix < G.wp:
                            s += w * P[k, iy, ix]
                    Q += T * s[:3]
                    T *= 1 - s[3]
                assert np.allclose(out[v, y, x], [*Q, T], atol=1e-13)


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_composite_at_matches_full(interp):
    p = _planes(4, G.hp, G.wp, 8, depth_range=(G.d_forward + 0.3, 7.0))
    out, _ = composite.composite(p["rgba"], p["depth"], CAM, G, DX32, DY32, interp)
    rng = np.random.default_rng(0)
    pix = np.stack([rng.integers(0, 5, 200), rng.integers(0, G.ny, 200), rng.integers(0, G.nx, 200)], 1)
    P = p["rgba"].astype(np.float64)
    f = lambda k, iy, ix: (P[k, iy, ix], np.zeros(iy.size, bool))
    at, _ = composite.composite_at(f, p["depth"], CAM, G, DX32, DY32, interp, pix)
    assert np.allclose(at, out[pix[:, 0], pix[:, 1], pix[:, 2]], atol=1e-14)
