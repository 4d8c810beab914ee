"""Pins of the spherical-harmonic oracle (the SH ablation of Fig. 6) to things other than
itself: SciPy's complex spherical harmonics, orthonormality on the sphere, the RGB oracle
(degree 0 and per-coefficient linearity), Eq. 5's principal rays and Eq. 6's reference
texels."""
import math

import numpy as np
import pytest
import scipy.special

import scenegen
from oracle import composite, decisions, geometry, render, sh, splat


def _unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


def test_basis_matches_scipy_real_combination():
    """Y_l0 = Y_l^0, Y_lm = sqrt(2) Re Y_l^m (m > 0), sqrt(2) Im Y_l^|m| (m < 0), with SciPy's
    Condon-Shortley-phased complex harmonics."""
    d = _unit(np.random.default_rng(0), 64)
    polar = np.arccos(np.clip(d[:, 2], -1, 1))
    azim = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
    got = sh.basis(d, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            c = scipy.special.sph_harm_y(l, abs(m), polar, azim)
            ref = c.real if m == 0 else math.sqrt(2) * (c.real if m > 0 else c.imag)
            np.testing.assert_allclose(got[:, l * l + l + m], ref, atol=1e-12, err_msg=f"l={l} m={m}")


def test_basis_orthonormal_on_the_sphere():
    """Gauss-Legendre in cos(polar) x uniform azimuth integrates the degree <= 6 products exactly."""
    z, wz = np.polynomial.legendre.leggauss(8)
    phi = np.arange(16) * (2 * np.pi / 16)
    Z, P = np.meshgrid(z, phi, indexing="ij")
    r = np.sqrt(1 - Z * Z)
    d = np.stack([r * np.cos(P), r * np.sin(P), Z], axis=-1).reshape(-1, 3)
    w = (wz[:, None] * np.full(16, 2 * np.pi / 16)[None, :]).reshape(-1)
    Y = sh.basis(d, 3)
    np.testing.assert_allclose((Y * w[:, None]).T @ Y, np.eye(16), atol=1e-12)


def test_gaussian_colour_closed_forms():
    Y10 = math.sqrt(3 / (4 * math.pi))
    c = np.zeros((3, 16, 3))
    c[:, 2, 0] = 1.0                 # red: Y_1,0 = Y10 z
    c[2, 2, 0] = -2.0                # third: clamped at zero along +z
    d = np.array([[0, 0, 1.0], [1.0, 0, 0], [0, 0, 1.0]])
    got = sh.gaussian_colour(c, d, 3)
    np.testing.assert_allclose(got[:, 0], [Y10 + 0.5, 0.5, 0.0], atol=1e-15)
    np.testing.assert_allclose(got[:, 1:], 0.5, atol=1e-15)


def test_image_centres_look_at_the_focal_plane_centre():
    """Eq. 5 shifts each view's principal point so that its frustum stays centred on the focal
    plane: the ray through the image centre of view (dx, dy) passes the focal-plane centre."""
    R = _rotation(3)
    cam = scenegen.camera(96, 64, 50.0, 2.5, math.radians(30), math.radians(10), R=R, t=[0.1, -0.2, 0.3])
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    g = geometry.derive(cam)
    for dx, dy in [(0.0, 0.0), (0.3, -0.1), (-0.25, 0.2)]:
        d = sh.pixel_directions(cam, g, dx, dy, [g.cx], [g.cy])[0, 0]
        t = np.asarray(cam.t, np.float64)
        to_centre = R.T @ (np.array([0.0, 0.0, g.d_focal]) - t) - sh.camera_centre(cam, dx, dy)
        np.testing.assert_allclose(d, to_centre / np.linalg.norm(to_centre), atol=1e-12)


def test_pixel_rays_pass_their_reference_texels():
    """Eq. 6 maps view pixel (x, y) to the reference texel its ray crosses on plane k: the
    point back-projected from that texel lies on the pixel's ray."""
    R = _rotation(5)
    cam = scenegen.camera(80, 60, 50.0, 2.0, math.radians(40), math.radians(16), R=R, t=[0.0, 0.1, -0.2])
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    g = geometry.derive(cam)
    depth = np.array([g.d_forward + 0.5, 2.0, 7.5], np.float32)
    dx = np.array([-0.3, 0.2], np.float32)
    dy = np.array([0.1, -0.15], np.float32)
    c = decisions.constants(g, cam)
    pc = decisions.plane_coeffs32(c, depth, dx, dy)
    xs, ys = np.array([0, 17, 79]), np.array([0, 31, 59])
    for v in range(2):
        d = sh.pixel_directions(cam, g, float(dx[v]), float(dy[v]), xs, ys)
        for k in range(3):
            X, Y = decisions.texel_coords32(pc, c, k, v, xs, ys, nearest=False)
            zr = float(depth[k]) - g.d_forward
            P = np.stack(np.broadcast_arrays((X[None, :].astype(np.float64) - g.cpx) / g.fpx * zr,
                                             (Y[:, None].astype(np.float64) - g.cpy) / g.fpy * zr,
                                             np.full((3, 3), float(depth[k]))), axis=-1)
            ray = (P - np.array([dx[v], dy[v], 0.0])) @ R
            ray /= np.linalg.norm(ray, axis=-1, keepdims=True)
            np.testing.assert_allclose(ray, d, atol=2e-5)


def _scene_sh(n, seed, degree):
    scene = scenegen.small_scene(n, seed)
    coef = scenegen.sh_coefficients(n, degree, seed + 1)
    if degree == 0:                  # rgb = the view-independent colour sh_0 Y_0 + 1/2 (>= 0)
        scene["rgb"] = sh.gaussian_colour(coef, np.tile([0.0, 0.0, 1.0], (n, 1)), 0)
    return scene, coef


def test_degree0_planes_and_views_equal_rgb():
    """Degree 0: q_0 Y_0 + A/2 is the plane colour of rgb = sh_0 Y_0 + 1/2, and the SH
    composite is the RGB composite (the clamp is inactive for rgb >= 0)."""
    scene, coef = _scene_sh(120, 2, 0)
    cam = scenegen.camera(40, 32, 50.0, 3.0, math.radians(30), math.radians(8))
    K = 3
    q, A, amb, depth = sh.build_sh_planes(scene, coef, 0, cam, K)
    rgb = render.build_mpi_gaussians(scene, cam, K)
    Y0 = 0.5 / math.sqrt(math.pi)
    np.testing.assert_allclose(q[..., 0, :] * Y0 + 0.5 * A[..., None], rgb.planes[..., :3], atol=1e-12)
    np.testing.assert_allclose(A, rgb.planes[..., 3], atol=1e-15)
    g = geometry.derive(cam)
    dx, dy, _, _ = geometry.quilt_views(cam, 3, 2)
    dx, dy = dx.astype(np.float32), dy.astype(np.float32)
    for interp in ("nearest", "bilinear"):
        got = sh.composite_sh(q, A, 0, depth, cam, g, dx, dy, interp)
        ref, _ = composite.composite(rgb.planes, depth, cam, g, dx, dy, interp)
        np.testing.assert_allclose(got, ref, atol=1e-12)


def test_sh_planes_blend_each_coefficient_like_rgb():
    """Coefficient j of the SH planes is the RGB oracle's plane colour for rgb := sh[:, j]."""
    scene, coef = _scene_sh(80, 4, 3)
    cam = scenegen.camera(32, 32, 50.0, 3.0, math.radians(30))
    q, A, _, _ = sh.build_sh_planes(scene, coef, 3, cam, 2)
    for j in (0, 5, 15):
        alt = dict(scene)
        alt["rgb"] = coef[:, j, :]
        ref = render.build_mpi_gaussians(alt, cam, 2)
        np.testing.assert_allclose(q[..., j, :], ref.planes[..., :3], atol=1e-12)
        np.testing.assert_allclose(A, ref.planes[..., 3], atol=1e-15)


def test_composite_sh_of_one_plane_is_the_basis_sum():
    """One fully covered plane of constant texels: each pixel is max(sum_j q_j Y_j(d) + A/2, 0)
    with d the direction from the view camera to the pixel's point on the plane (Eq. 6)."""
    R = _rotation(9)
    cam = scenegen.camera(24, 20, 50.0, 2.0, math.radians(30), math.radians(10), R=R)
    R = np.asarray(cam.R, np.float64).reshape(3, 3)          # as stored (float32)
    g = geometry.derive(cam)
    rng = np.random.default_rng(1)
    qv = rng.normal(scale=0.3, size=(16, 3))
    q = np.broadcast_to(qv, (1, g.hp, g.wp, 16, 3)).copy()
    A = np.full((1, g.hp, g.wp), 0.7)
    depth = np.array([2.0], np.float32)
    dx, dy = np.array([0.2], np.float32), np.array([-0.1], np.float32)
    out = sh.composite_sh(q, A, 3, depth, cam, g, dx, dy, "nearest")[0]
    # pixel (x, y) of the view sees the focal plane z = 2 at a point on its ray; the ray's
    # direction from the view centre, through the pinhole model, in world axes
    xs, ys = np.arange(g.nx), np.arange(g.ny)
    cxv = g.cx + float(dx[0]) / (g.d_focal * g.tx) * g.nx / 2.0
    cyv = g.cy + float(dy[0]) / (g.d_focal * g.ty) * g.ny / 2.0
    for y in (0, 9, 19):
        for x in (0, 11, 23):
            p = np.array([(x - cxv) / g.fx, (y - cyv) / g.fy, 1.0]) @ R
            d = p / np.linalg.norm(p)
            Y = sh.basis(d[None], 3)[0]
            want = np.maximum(Y @ qv + 0.35, 0.0)
            np.testing.assert_allclose(out[y, x, :3], want, atol=1e-12)
            assert abs(out[y, x, 3] - 0.3) < 1e-15


def test_render_view_sh_degree0_equals_rgb_render():
    scene, coef = _scene_sh(100, 6, 0)
    cam = scenegen.camera(32, 24, 50.0, 3.0, math.radians(30))
    got, _ = sh.render_view_sh(scene, coef, 0, cam, 0.1, -0.05)
    ref, _ = render.render_view(scene, cam, 0.1, -0.05)
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_view_colours_use_the_view_centre():
    """A Gaussian straight ahead of a view camera is seen along that camera's z axis."""
    R = _rotation(2)
    cam = scenegen.camera(32, 32, 50.0, 2.0, math.radians(30), R=R, t=[0.2, 0.1, -0.3])
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    centre = sh.camera_centre(cam, 0.3, -0.2)
    axis = R.T @ np.array([0.0, 0.0, 1.0])
    scene = {"means": (centre + 2.5 * axis)[None]}
    coef = np.zeros((1, 4, 3))
    coef[0, 1:, 0] = [0.4, -0.7, 0.2]
    got = sh.view_colours(scene, coef, 1, cam, 0.3, -0.2)
    Y = sh.basis(axis[None], 1)[0]
    np.testing.assert_allclose(got[0], [max(Y[1:] @ [0.4, -0.7, 0.2] + 0.5, 0.0), 0.5, 0.5], atol=1e-12)


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_basis_degree_prefix(degree):
    d = _unit(np.random.default_rng(7), 9)
    np.testing.assert_array_equal(sh.basis(d, degree), sh.basis(d, 3)[:, :sh.n_coef(degree)])


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_composite_sh_at_matches_whole_views(interp):
    """The per-pixel SH composite (used at full size) equals the whole-view one."""
    R = np.asarray(_rotation(8))
    cam = scenegen.camera(40, 30, 50.0, 2.0, math.radians(30), math.radians(10), R=R)
    g = geometry.derive(cam)
    rng = np.random.default_rng(2)
    K, nc = 3, 9
    A = rng.uniform(0, 0.8, (K, g.hp, g.wp))
    q = rng.normal(scale=0.3, size=(K, g.hp, g.wp, nc, 3)) * A[..., None, None]
    depth = np.sort(rng.uniform(g.d_forward + 0.3, 8.0, K)).astype(np.float32)
    dx, dy, _, _ = geometry.quilt_views(cam, 3, 2)
    dx, dy = dx.astype(np.float32), dy.astype(np.float32)
    full = sh.composite_sh(q, A, 2, depth, cam, g, dx, dy, interp)
    stacked = np.concatenate([q.reshape(K, g.hp, g.wp, 3 * nc), A[..., None]], axis=-1)
    f = lambda k, iy, ix: (stacked[k, iy, ix], np.zeros(iy.size, bool))
    pix = np.stack([rng.integers(0, 6, 150), rng.integers(0, g.ny, 150), rng.integers(0, g.nx, 150)], 1)
    at, _ = sh.composite_sh_at(f, 2, depth, cam, g, dx, dy, interp, pix)
    np.testing.assert_allclose(at, full[pix[:, 0], pix[:, 1], pix[:, 2]], atol=1e-13)
