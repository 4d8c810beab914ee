"""Pins of the sparse-voxel oracle (Sec. 4.5) against closed forms, an independent
quadrature, brute-force ray marching and the filter's impulse response."""
import math

import numpy as np
import pytest
from scipy import integrate

import scenegen
from oracle import geometry, voxels


def _cam(res=33, d_focal=3.0, phi=0.0, fov=50.0):
    return scenegen.camera(res, res, fov, d_focal, phi, 0.0)


def _one_voxel(ijk, dens, rgb, origin=(-1.0, -1.0, 3.0), h=1.0 / 16):
    return dict(ijk=np.asarray([ijk], dtype=np.int32), density=np.asarray([dens], dtype=np.float32),
                rgb=np.asarray([rgb], dtype=np.float32), origin=origin, voxel_size=h)


def test_centres_float32_program():
    ijk = np.array([[0, 1, 2], [255, 128, 7]], dtype=np.int32)
    c = voxels.centres32(ijk, (-1.0, -1.0, 3.0), 2.0 / 256)
    assert c.dtype == np.float32
    exact = np.array([-1.0, -1.0, 3.0]) + (2.0 / 256) * (ijk + 0.5)
    assert np.abs(c - exact).max() < 4e-7


def test_constant_density_axial_ray_closed_form():
    """A constant-density voxel centred on the optical axis: the principal texel's ray runs
    along +z through both z faces, so tau = rho h and alpha = 1 - exp(-rho h)."""
    cam = _cam()
    g = geometry.derive(cam)
    assert g.cpx == 16.0 and g.cpy == 16.0
    h, rho = 1.0 / 16, 7.5
    vox = _one_voxel((0, 0, 0), [rho] * 8, [0.2, 0.5, 0.9], origin=(-h / 2, -h / 2, 4.0), h=h)
    plane = voxels.render_plane(vox, np.array([0]), cam, g)
    alpha = 1.0 - math.exp(-rho * h)
    np.testing.assert_allclose(plane[16, 16, 3], alpha, rtol=1e-12)
    np.testing.assert_allclose(plane[16, 16, :3], alpha * np.array([0.2, 0.5, 0.9]), rtol=1e-6)


def test_constant_density_oblique_chord():
    """Oblique ray through the front and back faces: chord = h |r| / r_z with r_z = 1."""
    cam = _cam()
    g = geometry.derive(cam)
    h, rho = 0.5, 2.0
    z0 = 4.0
    # the ray of texel (18, 16) at the voxel's mid depth sits at x = (2 / f'_x) (z - D_fwd)
    xm = (2.0 / g.fpx) * (z0 + h / 2 - g.d_forward)
    vox = _one_voxel((0, 0, 0), [rho] * 8, [1, 1, 1], origin=(xm - h / 2, -h / 2, z0), h=h)
    plane = voxels.render_plane(vox, np.array([0]), cam, g)
    r = np.array([2.0 / g.fpx, 0.0, 1.0])
    # x stays inside the voxel over the z extent: |r_x| h / 2 << h / 2
    assert abs(r[0]) * h / 2 < h / 2
    np.testing.assert_allclose(plane[16, 18, 3], 1.0 - math.exp(-rho * h * np.linalg.norm(r)), rtol=1e-12)


def test_linear_density_along_ray():
    """Density varying only with z: tau along the axis = h (rho_front + rho_back) / 2."""
    cam = _cam()
    g = geometry.derive(cam)
    h = 0.25
    dens = [3.0 if (c >> 2) & 1 == 0 else 11.0 for c in range(8)]
    vox = _one_voxel((0, 0, 0), dens, [1, 0, 0], origin=(-h / 2, -h / 2, 4.0), h=h)
    plane = voxels.render_plane(vox, np.array([0]), cam, g)
    np.testing.assert_allclose(plane[16, 16, 3], 1.0 - math.exp(-h * 7.0), rtol=1e-12)


def test_optical_depth_matches_adaptive_quadrature():
    """The Gauss-Legendre line integral equals scipy's adaptive quadrature of the trilinear
    density (an independent integrator) on random voxels and rays."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        dens = rng.uniform(0.1, 50.0, 8)
        a = rng.uniform(-0.5, 1.5, 3)
        b = rng.normal(size=3)
        t0, t1 = voxels.slab(a[None], b[None])
        if not t1[0] > t0[0]:
            continue
        rn = np.array([1.7])

        def rho(t):
            u = a + t * b
            return sum(dens[c] * np.prod([u[ax] if (c >> ax) & 1 else 1 - u[ax] for ax in range(3)]) for c in range(8))
        ref, _ = integrate.quad(rho, t0[0], t1[0], epsabs=1e-13, epsrel=1e-13)
        got = voxels.optical_depth(dens, a[None], b[None], rn)[0]
        np.testing.assert_allclose(got, 1.7 * ref, rtol=1e-10)


def test_two_point_rule_is_exact_for_the_trilinear_line_integral():
    """The trilinear density along a line is a cubic in t, so a 2-point Gauss-Legendre rule
    (the kernel's) integrates it exactly; pin that against the oracle's 3-point rule."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        dens = rng.uniform(0.1, 50.0, 8)
        a, b = rng.uniform(0.0, 1.0, 3), rng.normal(size=3)
        t0, t1 = voxels.slab(a[None], b[None])
        mid, half = 0.5 * (t0[0] + t1[0]), 0.5 * (t1[0] - t0[0])
        g2 = half * sum(voxels.trilinear(dens, a + (mid + half * s) * b) for s in (-1 / math.sqrt(3), 1 / math.sqrt(3)))
        g3 = voxels.optical_depth(dens, a[None], b[None], np.ones(1))[0]
        np.testing.assert_allclose(g2, g3, rtol=1e-12)


def test_slab_interval_brute_force():
    rng = np.random.default_rng(11)
    for _ in range(50):
        a, b = rng.uniform(-1.0, 2.0, 3), rng.normal(size=3)
        t0, t1 = voxels.slab(a[None], b[None])
        ts = np.linspace(0.0, 6.0, 60001)
        inside = np.all((a[None] + ts[:, None] * b[None] >= 0) & (a[None] + ts[:, None] * b[None] <= 1), axis=1)
        if not inside.any():
            assert not (t1[0] > t0[0] and t0[0] < 6.0 - 1e-3 and t1[0] - t0[0] > 2e-4)
            continue
        np.testing.assert_allclose(ts[inside].min(), t0[0], atol=2e-4)
        np.testing.assert_allclose(ts[inside].max(), min(t1[0], 6.0), atol=2e-4)


def test_plane_matches_ray_marching_brute_force():
    """A tiny random scene: per texel, march each voxel of the chunk in its blending order
    with a fine midpoint rule (independent of the slab and quadrature code)."""
    vox = scenegen.voxel_scene(res=8, n_occupied=40, seed=5, bbox=((-0.6, -0.6, 2.8), (0.6, 0.6, 4.0)))
    vox["density"] = vox["density"] * np.float32(0.03)        # semi-transparent voxels
    cam = _cam(res=24, d_focal=3.0)
    g = geometry.derive(cam)
    part = voxels.partition_voxels(vox, cam, g, 1)
    idx = part.order
    plane = voxels.render_plane(vox, idx, cam, g)
    h = vox["voxel_size"]
    o = np.array([0.0, 0.0, g.d_forward])
    a = plane[..., 3]
    partial = np.argwhere((a > 0.02) & (a < 0.98))
    assert len(partial) >= 8
    picks = [tuple(p) for p in partial[np.random.default_rng(0).choice(len(partial), 8, replace=False)]]
    picks += [tuple(p) for p in np.argwhere(a == 0.0)[:2]]
    for (py, px) in picks:
        r = np.array([(px - g.cpx) / g.fpx, (py - g.cpy) / g.fpy, 1.0])
        C, T = np.zeros(3), 1.0
        ts = (np.arange(40000) + 0.5) * (4.0 / 40000)
        dt = 4.0 / 40000
        pts = o + ts[:, None] * r
        for i in idx:
            lo = np.asarray(vox["origin"]) + h * vox["ijk"][i]
            u = (pts - lo) / h
            m = np.all((u >= 0) & (u <= 1), axis=1)
            if not m.any():
                continue
            tau = np.linalg.norm(r) * dt * voxels.trilinear(vox["density"][i].astype(np.float64), u[m]).sum()
            al = 1 - math.exp(-tau)
            C += T * al * vox["rgb"][i]
            T *= 1 - al
        np.testing.assert_allclose(plane[py, px, :3], C, atol=2e-4)
        np.testing.assert_allclose(plane[py, px, 3], 1 - T, atol=2e-4)


def test_two_voxels_front_to_back_order():
    cam = _cam()
    g = geometry.derive(cam)
    h = 0.2
    vox = dict(ijk=np.array([[0, 0, 0], [0, 0, 3]], dtype=np.int32),
               density=np.array([[4.0] * 8, [9.0] * 8], dtype=np.float32),
               rgb=np.array([[1, 0, 0], [0, 0, 1]], dtype=np.float32), origin=(-h / 2, -h / 2, 4.0), voxel_size=h)
    a1, a2 = 1 - math.exp(-4.0 * h), 1 - math.exp(-9.0 * h)
    fwd = voxels.render_plane(vox, np.array([0, 1]), cam, g)[16, 16]
    np.testing.assert_allclose(fwd, [a1, 0, (1 - a1) * a2, 1 - (1 - a1) * (1 - a2)], rtol=1e-6)
    rev = voxels.render_plane(vox, np.array([1, 0]), cam, g)[16, 16]
    np.testing.assert_allclose(rev, [(1 - a2) * a1, 0, a2, 1 - (1 - a1) * (1 - a2)], rtol=1e-6)


def test_support_rect_contains_every_hit_texel():
    vox = scenegen.voxel_scene(res=8, n_occupied=30, seed=9, bbox=((-0.6, -0.6, 2.8), (0.6, 0.6, 4.0)))
    cam = _cam(res=24)
    g = geometry.derive(cam)
    h = vox["voxel_size"]
    ys, xs = np.meshgrid(np.arange(g.hp, dtype=np.float64), np.arange(g.wp, dtype=np.float64), indexing="ij")
    r = voxels.texel_rays(g, xs, ys)
    for i in range(30):
        lo = np.asarray(vox["origin"], dtype=np.float64) + h * vox["ijk"][i]
        a = np.broadcast_to((np.array([0.0, 0.0, g.d_forward]) - lo) / h, r.shape)
        t0, t1 = voxels.slab(a, r / h)
        hit = t1 > t0
        x0, y0, x1, y1 = voxels.support_rect(lo, h, cam, g)
        yy, xx = np.nonzero(hit)
        assert hit.any()
        assert xx.min() >= x0 and xx.max() <= x1 and yy.min() >= y0 and yy.max() <= y1


def test_lowpass_impulse_response_and_constants():
    p = np.zeros((7, 9, 2))
    p[3, 4, 0] = 1.0
    out = voxels.lowpass(p)
    k = np.outer([1, 2, 1], [1, 2, 1]) / 16.0
    np.testing.assert_allclose(out[2:5, 3:6, 0], k, rtol=0, atol=1e-15)
    assert abs(out[..., 0].sum() - 1.0) < 1e-15
    c = np.full((6, 5, 1), 0.37)
    oc = voxels.lowpass(c)
    np.testing.assert_allclose(oc[1:-1, 1:-1], 0.37, rtol=1e-15)
    np.testing.assert_allclose(oc[0, 2], 0.37 * 0.75, rtol=1e-15)       # zero padding above
    np.testing.assert_allclose(oc[0, 0], 0.37 * 0.75 * 0.75, rtol=1e-15)


def test_build_mpi_voxels_partition_uses_centre_keys():
    vox = scenegen.voxel_scene(res=16, n_occupied=200, seed=4, bbox=((-0.8, -0.8, 2.5), (0.8, 0.8, 4.1)))
    cam = _cam(res=24)
    mpi = voxels.build_mpi_voxels(vox, cam, 4, chunks=[0, 3])
    c = voxels.centres32(vox["ijk"], vox["origin"], vox["voxel_size"])
    keys = c[mpi.part.order, 2]
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)
    assert mpi.planes[1].max() == 0.0 and mpi.planes[0][..., 3].max() > 0.0
    a = mpi.planes[0][..., 3]
    assert a.min() >= 0.0 and a.max() <= 1.0


@pytest.mark.parametrize("res", [16])
def test_voxel_scene_recipe(res):
    vox = scenegen.voxel_scene(res=res, n_occupied=50, seed=1)
    assert vox["ijk"].dtype == np.int32 and vox["ijk"].shape == (50, 3)
    assert (vox["ijk"] >= 0).all() and (vox["ijk"] < res).all()
    lin = (vox["ijk"][:, 2] * res + vox["ijk"][:, 1]) * res + vox["ijk"][:, 0]
    assert np.all(np.diff(lin) > 0)
