"""Pins of the oracle's display geometry (Sec. 4.2-4.3, Eqs. 1-6, 8) against closed forms
and an independent ray-casting construction."""
import json
import math
import os

import numpy as np
import pytest

import scenegen
from oracle import decisions, geometry

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cam(**kw):
    base = dict(nx=256, ny=192, fov_deg=50.0, d_focal=2.0, phi_x=math.radians(40.0), phi_y=0.0)
    base.update(kw)
    return scenegen.camera(**base)


def test_golden_closed_forms():
    """Hand-derived cases (tests/golden/geometry_closed_forms.json)."""
    with open(os.path.join(GOLDEN, "geometry_closed_forms.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        cam = scenegen.camera(c["nx"], c["ny"], c["fov_deg"], c["d_focal"], math.radians(c["phi_x_deg"]),
                              math.radians(c["phi_y_deg"]), plane_scale=c["plane_scale"],
                              d_shift=c["d_shift"])
        g = geometry.derive(cam)
        tx = math.tan(0.5 * cam.fov_x)
        exp = c["expect"]
        assert g.d_forward0 == pytest.approx(exp["d_forward_over_d_focal"] * cam.d_focal, rel=1e-12)
        assert g.tpx == pytest.approx(exp["tan_half_theta_prime_over_tan_half_theta"] * tx, rel=1e-12)
        assert g.f_dilation == pytest.approx(exp["f_dilation"], rel=1e-12)
        assert (g.wp, g.hp) == tuple(exp["plane_wh"])


@pytest.mark.parametrize("phi_deg,fov_deg", [(5.0, 50.0), (40.0, 50.0), (70.0, 30.0), (10.0, 90.0)])
def test_reference_cone_is_tangent_to_outermost_view(phi_deg, fov_deg):
    """Eqs. 1-2 place the reference frustum edge on the outermost view's window-edge ray.

    The outermost view sits at dx = D_f tan(phi/2) (Eqs. 3-4) and its frustum passes
    through the window edges at the focal plane; the reference edge through the same
    window edge must have the same slope, so tan(theta'/2) = tan(theta/2) + tan(phi/2).
    Behind the focal plane every view ray stays inside the reference frustum.
    """
    cam = _cam(fov_deg=fov_deg, phi_x=math.radians(phi_deg))
    g = geometry.derive(cam)
    assert g.tpx == pytest.approx(g.tx + g.taux, rel=1e-12)
    dx, _, px, _ = geometry.quilt_views(cam, 9, 1)
    z = np.linspace(g.d_focal, 50 * g.d_focal, 200)
    for dxv, pv in zip(dx, px):
        for u in (-1.0, 1.0):
            x = dxv + z * g.tx * (u - pv)          # ray of view pixel NDC u (shifted principal point)
            assert np.all(np.abs(x) <= g.tpx * (z - g.d_forward) * (1 + 1e-12) + 1e-12)


def test_zero_viewing_angle_and_fov_growth():
    cam0 = _cam(phi_x=0.0)
    g0 = geometry.derive(cam0)
    assert g0.d_forward == 0.0
    assert g0.tpx == pytest.approx(g0.tx, rel=1e-15)
    for phi in (1.0, 10.0, 60.0):
        g = geometry.derive(_cam(phi_x=math.radians(phi)))
        assert g.d_forward > 0 and g.tpx > g.tx and g.tpy > g.ty


@pytest.mark.parametrize("shift,ps", [(0.0, 1.0), (0.0, 2.0), (0.3, 1.0), (0.5, 3.0)])
def test_adaptive_dilation_closed_form(shift, ps):
    """Eq. 8 with theta' fixed before the shift: ratio = (D_f - D0)/(D_f - D0 + D_shift)."""
    cam = _cam(d_shift=shift, plane_scale=ps)
    g = geometry.derive(cam)
    ratio = (g.d_focal - g.d_forward0) / (g.d_focal - g.d_forward0 + cam.d_shift)
    assert g.f_dilation == pytest.approx(0.3 * (ratio * ps) ** 2, rel=1e-12)


@pytest.mark.parametrize("ps", [1.0, 2.0, 3.0])
def test_constant_dilation_overrides_eq8(ps):
    """A camera's constant dilation (the adaptive-filter ablation) replaces Eq. 8 whatever P_s;
    with no baseline and P_s = 1, Eq. 8 itself is the constant 0.3 of 3DGS."""
    g = geometry.derive(_cam(plane_scale=ps, dilation=float(np.float32(0.45))))
    assert g.f_dilation == float(np.float32(0.45))
    flat = scenegen.camera(64, 48, 50.0, 2.0, 0.0)
    assert geometry.derive(flat).f_dilation == pytest.approx(0.3, rel=1e-15)


def test_view_grid():
    cam = scenegen.config("uniform10k")[1]
    dx, dy, px, py = geometry.quilt_views(cam, 9, 1)
    assert dx[0] == pytest.approx(-0.05, rel=1e-6) and dx[-1] == pytest.approx(0.05, rel=1e-6)
    assert dx[-1] - dx[0] == pytest.approx(0.1, rel=1e-6)          # "baseline of 0.1"
    assert np.allclose(dx, -dx[::-1]) and np.all(dy == 0)
    g = geometry.derive(cam)
    # principal rays meet the focal-plane centre: dx - D_f tan(theta/2) p = 0
    assert np.allclose(dx - g.d_focal * g.tx * px, 0.0, atol=1e-15)
    dx1, _, _, _ = geometry.quilt_views(cam, 1, 1)
    assert dx1.tolist() == [0.0]


def _ray_cast_texel(g, dx, dy, px, py, d, x, y):
    """Texel hit on plane z=d by the ray of view pixel (x, y): camera matrices, no Eq. 6."""
    K = np.array([[g.fx, 0.0, g.cx + px * g.nx / 2.0], [0.0, g.fy, g.cy + py * g.ny / 2.0], [0, 0, 1.0]])
    dirs = np.linalg.solve(K, np.stack([x, y, np.ones_like(x)]))
    P = np.array([dx, dy, 0.0])[:, None] + dirs * (d / dirs[2])
    Kr = np.array([[g.fpx, 0.0, g.cpx], [0.0, g.fpy, g.cpy], [0, 0, 1.0]])
    h = Kr @ (P - np.array([0.0, 0.0, g.d_forward])[:, None])
    return h[0] / h[2], h[1] / h[2]


@pytest.mark.parametrize("phi_y_deg,ps", [(0.0, 1.0), (15.0, 2.0)])
def test_eq6_equals_ray_plane_intersection(phi_y_deg, ps):
    cam = _cam(phi_y=math.radians(phi_y_deg), plane_scale=ps)
    g = geometry.derive(cam)
    dxs, dys, pxs, pys = geometry.quilt_views(cam, 7, 3 if phi_y_deg else 1)
    rng = np.random.default_rng(3)
    x = rng.uniform(-0.5, g.nx - 0.5, 50)
    y = rng.uniform(-0.5, g.ny - 0.5, 50)
    for v in range(len(dxs)):
        for d in (g.d_forward + 0.2, 1.0, g.d_focal, 7.5, 40.0):
            X = geometry.ndc_to_texel(geometry.u_prime(g, dxs[v], d, geometry.pixel_ndc(x, g.nx)), g.wp)
            Y = geometry.ndc_to_texel(geometry.v_prime(g, dys[v], d, geometry.pixel_ndc(y, g.ny)), g.hp)
            Xr, Yr = _ray_cast_texel(g, dxs[v], dys[v], pxs[v], pys[v], d, x, y)
            assert np.allclose(X, Xr, rtol=0, atol=1e-9 * g.wp)
            assert np.allclose(Y, Yr, rtol=0, atol=1e-9 * g.hp)


def test_eq6_focal_plane_and_antisymmetry():
    cam = _cam()
    g = geometry.derive(cam)
    u = np.linspace(-1, 1, 11)
    for dx in (-0.3, 0.0, 0.41):
        assert np.allclose(geometry.u_prime(g, dx, g.d_focal, u), u, atol=1e-14)   # zero-parallax plane
        for d in (1.0, 3.3, 15.0):
            assert np.allclose(geometry.u_prime(g, -dx, d, -u), -geometry.u_prime(g, dx, d, u), atol=1e-14)


@pytest.mark.parametrize("name", ["uniform10k", "cluster500k"])
def test_fp32_coordinate_program_tracks_eq6(name):
    """The float32 texel-coordinate program agrees with float64 Eq. 6 to 2e-4 texel.

    Bound: about eight float32 roundings, each <= 2^-24 relative, of a coordinate at most
    W_p/2 + 2 texels from the plane centre, plus the rounding of D_forward, which the
    near planes (d - D_forward >= 0.2) magnify by at most D_forward / 0.2.
    """
    cam, cfg = scenegen.config_camera(name)
    g = geometry.derive(cam)
    c = decisions.constants(g, cam)
    dx, dy, _, _ = geometry.quilt_views(cam, cfg["vx"], cfg["vy"])
    dx32, dy32 = dx.astype(np.float32), dy.astype(np.float32)
    depth = np.geomspace(g.d_forward + 0.21, 25.0, 40).astype(np.float32)
    pc = decisions.plane_coeffs32(c, depth, dx32, dy32)
    xs = np.arange(g.nx)
    worst = 0.0
    for k in range(depth.size):
        for v in range(len(dx)):
            X, Y = decisions.texel_coords32(pc, c, k, v, xs, xs, nearest=False)
            Xe = geometry.ndc_to_texel(geometry.u_prime(g, float(dx32[v]), float(depth[k]),
                                                        geometry.pixel_ndc(xs, g.nx)), g.wp)
            Ye = geometry.ndc_to_texel(geometry.v_prime(g, float(dy32[v]), float(depth[k]),
                                                        geometry.pixel_ndc(xs, g.ny)), g.hp)
            inside = (Xe > -2) & (Xe < g.wp + 1)
            worst = max(worst, np.max(np.abs(X - Xe)[inside], initial=0.0), np.max(np.abs(Y - Ye)))
            Xn, _ = decisions.texel_coords32(pc, c, k, v, xs, xs, nearest=True)
            assert np.all(np.abs((Xn.astype(np.float64) - 0.5) - X) <= 1e-4)
    assert worst <= 2e-4, worst
