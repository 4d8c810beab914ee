"""Pins of the oracle's per-view render away from the reference axis (Sec. 4.3, Eq. 5).

A view of the quilt is a pinhole camera at (dx, dy, 0) in base-camera coordinates with the
base camera's orientation and focal lengths; Eq. 5 shifts its principal point so that its
principal ray meets the centre of the focal plane.  These tests fix that geometry from its
definition, not from the oracle's formula:

* a small Gaussian at the focal-plane centre renders centred on the image centre, for every
  view offset (a wrong sign of the shift, or of the camera position, moves it by p_x N_x);
* 1-3 Gaussians off the focal plane render centred where a 3x4 camera matrix built here by
  hand, P = K_v [R | t - (dx, dy, 0)], projects their means (parallax included).
"""
import math

import numpy as np
import pytest

import scenegen
from oracle import geometry, render


def _scene(means_world, log_sigma):
    n = len(means_world)
    return dict(means=np.asarray(means_world, np.float32),
                log_scales=np.full((n, 3), log_sigma, np.float32),
                quats=np.tile(np.array([1.0, 0.0, 0.0, 0.0], np.float32), (n, 1)),
                opacity=np.full(n, 0.9, np.float32), rgb=np.ones((n, 3), np.float32))


def _rotation(ax, ay, az):
    cx, sx, cy, sy, cz, sz = math.cos(ax), math.sin(ax), math.cos(ay), math.sin(ay), math.cos(az), math.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def _centroids(alpha, centres, radius):
    """Alpha-weighted centroid of the blob around each expected centre."""
    ys, xs = np.mgrid[0:alpha.shape[0], 0:alpha.shape[1]]
    out = []
    for cx, cy in centres:
        w = alpha * ((xs - cx) ** 2 + (ys - cy) ** 2 <= radius ** 2)
        assert w.sum() > 1.0, "no blob near the expected position"
        out.append(((w * xs).sum() / w.sum(), (w * ys).sum() / w.sum()))
    return np.array(out)


def _to_world(R, t, p_cam):
    """World point whose base-camera coordinates are p_cam (p_cam = R X + t)."""
    return (np.asarray(p_cam, np.float64) - t) @ R


@pytest.mark.parametrize("dx,dy", [(0.0, 0.0), (0.2, 0.0), (-0.15, 0.1), (0.1, -0.2), (0.25, 0.25)])
def test_focal_plane_centre_renders_at_image_centre(dx, dy):
    cam = scenegen.camera(64, 48, 50.0, 2.0, math.radians(40.0), math.radians(30.0),
                          R=_rotation(0.1, -0.2, 0.05), t=(0.1, -0.05, 0.3))
    g = geometry.derive(cam)
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64)
    # screen sigma about 2 px at the focal plane
    sigma = 2.0 * g.d_focal / g.fx
    scene = _scene([_to_world(R, t, (0.0, 0.0, g.d_focal))], math.log(sigma))
    rgba, _ = render.render_view(scene, cam, dx, dy)
    c = _centroids(rgba[..., 3], [((cam.nx - 1) / 2, (cam.ny - 1) / 2)], 12.0)[0]
    assert abs(c[0] - (cam.nx - 1) / 2) < 0.02 and abs(c[1] - (cam.ny - 1) / 2) < 0.02, (dx, dy, c)


@pytest.mark.parametrize("dx,dy", [(0.0, 0.0), (0.3, 0.0), (-0.2, 0.15)])
def test_views_match_a_hand_built_camera_matrix(dx, dy):
    cam = scenegen.camera(96, 64, 45.0, 3.0, math.radians(40.0), math.radians(30.0),
                          R=_rotation(-0.15, 0.1, 0.2), t=(-0.2, 0.1, 0.5))
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64)
    fx = 0.5 * cam.nx / math.tan(0.5 * cam.fov_x)
    fy = 0.5 * cam.ny / math.tan(0.5 * cam.fov_y)
    # the view's principal point from the requirement itself: the focal-plane centre, at
    # (-dx, -dy, D_focal) in view coordinates, projects to the image centre
    D = cam.d_focal
    cxv = (cam.nx - 1) / 2 + fx * dx / D
    cyv = (cam.ny - 1) / 2 + fy * dy / D
    K = np.array([[fx, 0.0, cxv], [0.0, fy, cyv], [0.0, 0.0, 1.0]])
    P = K @ np.hstack([R, (t - np.array([dx, dy, 0.0]))[:, None]])
    # three Gaussians in front of, on and behind the focal plane, apart on the screen
    cam_pts = [(-0.35, -0.2, 1.6), (0.05, 0.15, 3.0), (0.9, -0.3, 5.5)]
    world = [_to_world(R, t, p) for p in cam_pts]
    scene = _scene(world, math.log(0.02))
    rgba, _ = render.render_view(scene, cam, dx, dy)
    proj = []
    for X in world:
        h = P @ np.append(X, 1.0)
        proj.append((h[0] / h[2], h[1] / h[2]))
    c = _centroids(rgba[..., 3], proj, 6.0)
    assert np.abs(c - np.array(proj)).max() < 0.02, (c, proj)
