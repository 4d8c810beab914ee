"""View-dependent colour in the sweeping planes: spherical harmonics (test infrastructure: oracle).

The paper's SH ablation (Sec. 5, Fig. 6) blends planes that keep view-dependent colour
instead of RGB.  This module states that variant in float64:

* Colour of a Gaussian.  Gaussian i carries real spherical-harmonic coefficients
  sh_i [n_coef, 3], n_coef = (L + 1)^2 for degree L <= 3, index j = l^2 + l + m.  Seen along
  the unit direction d its colour is max(sum_j sh_ij Y_j(d) + 1/2, 0) per channel (the
  convention of 3D Gaussian splatting, whose DC term carries the offset 1/2).
* SH planes.  A plane is shared by every view, so a texel cannot hold one colour.  It keeps
  the coefficients blended with the weights of the RGB planes (Alg. 1 "Rasterize"):
  q_j = sum_i alpha_i T_i sh_ij, and A = 1 - T.
* Compositing.  View v samples plane k at its pixel (x, y) exactly as the RGB composite does
  (Eq. 6, nearest or bilinear, applied to q and A), and the sample contributes the
  premultiplied colour max(sum_j q_j Y_j(d) + A / 2, 0), with d the direction of the
  pixel's ray in view v, the same for every plane along the ray; then Eq. 7 as for RGB.
  Blending is linear in the colour, so without the clamp this equals blending the
  Gaussians' own colours evaluated along d.  The clamp at zero can only act on the blended
  sum, not on each Gaussian (a reading; the paper does not say where its SH path clamps).
* The per-view render with SH colour evaluates each Gaussian along the direction from the
  view camera's centre to its mean, as 3D Gaussian splatting does, and rasterises as the
  RGB per-view render does.

Basis.  Real spherical harmonics with the Condon-Shortley phase, in the sign convention of
3D Gaussian splatting: Y_l0 = Y_l^0, Y_lm = sqrt(2) Re Y_l^m for m > 0 and
sqrt(2) Im Y_l^|m| for m < 0, written out as polynomials of the unit vector (x, y, z).
"""
from __future__ import annotations

import math

import numpy as np

from . import composite, decisions, geometry, partition, project, render, splat

MAX_DEGREE = 3


def n_coef(degree: int) -> int:
    return (degree + 1) ** 2


def basis(d, degree: int) -> np.ndarray:
    """Y_j(d) for j < (degree + 1)^2 at unit directions d [..., 3]; returns [..., n_coef]."""
    if not 0 <= degree <= MAX_DEGREE:
        raise ValueError(f"SH degree {degree} outside [0, {MAX_DEGREE}]")
    d = np.asarray(d, dtype=np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    pi = math.pi
    out = [np.full(x.shape, 0.5 / math.sqrt(pi))]
    if degree >= 1:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        out += [-c1 * y, c1 * z, -c1 * x]
    if degree >= 2:
        a = 0.5 * math.sqrt(15.0 / pi)
        b = 0.25 * math.sqrt(5.0 / pi)
        out += [a * x * y, -a * y * z, b * (2.0 * z * z - x * x - y * y), -a * x * z, 0.5 * a * (x * x - y * y)]
    if degree >= 3:
        e = 0.25 * math.sqrt(35.0 / (2.0 * pi))
        f = 0.5 * math.sqrt(105.0 / pi)
        g = 0.25 * math.sqrt(21.0 / (2.0 * pi))
        h = 0.25 * math.sqrt(7.0 / pi)
        w = 4.0 * z * z - x * x - y * y
        out += [-e * y * (3.0 * x * x - y * y), f * x * y * z, -g * y * w,
                h * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y), -g * x * w, 0.5 * f * z * (x * x - y * y),
                -e * x * (x * x - 3.0 * y * y)]
    return np.stack(out, axis=-1)


def gaussian_colour(sh, d, degree: int) -> np.ndarray:
    """max(sum_j sh_j Y_j(d) + 1/2, 0): sh [n, n_coef, 3], d [n, 3] unit -> [n, 3]."""
    Y = basis(d, degree)
    return np.maximum(np.einsum("nj,njc->nc", Y, np.asarray(sh, np.float64)[:, :n_coef(degree)]) + 0.5, 0.0)


def camera_centre(cam, dx: float = 0.0, dy: float = 0.0) -> np.ndarray:
    """World position of the view camera at lateral offset (dx, dy) in base-camera axes."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64)
    return R.T @ (np.array([dx, dy, 0.0]) - t)


def view_colours(scene: dict, sh, degree: int, cam, dx: float = 0.0, dy: float = 0.0) -> np.ndarray:
    """Every Gaussian's colour seen from the view camera at (dx, dy): direction centre -> mean."""
    v = np.asarray(scene["means"], np.float64) - camera_centre(cam, dx, dy)[None]
    return gaussian_colour(sh, v / np.linalg.norm(v, axis=1, keepdims=True), degree)


def pixel_directions(cam, g: geometry.Geometry, dx: float, dy: float, xs, ys) -> np.ndarray:
    """World unit directions [len(ys), len(xs), 3] of the pixel rays of view (dx, dy): the view
    camera has the base camera's axes and focal lengths and the principal point of Eq. 5,
    c_x = (N_x - 1)/2 + p_x N_x / 2, p_x = dx / (D_focal tan(theta_x / 2))."""
    cxv = g.cx + dx / (g.d_focal * g.tx) * g.nx / 2.0
    cyv = g.cy + dy / (g.d_focal * g.ty) * g.ny / 2.0
    xs = np.asarray(xs, np.float64)
    ys = np.asarray(ys, np.float64)
    rc = np.stack(np.broadcast_arrays((xs[None, :] - cxv) / g.fx, (ys[:, None] - cyv) / g.fy,
                                      np.ones((len(ys), len(xs)))), axis=-1)
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    w = rc @ R                                          # R^T applied to each camera-space ray
    return w / np.linalg.norm(w, axis=-1, keepdims=True)


def composite_sh_at(texel_fn, degree: int, depth32, cam, g: geometry.Geometry, dx32, dy32, interp: str, pix):
    """The SH composite at individual pixels pix [n,3] of (view, y, x).  texel_fn(k, iy, ix)
    returns (texels [m, 3 n_coef + 1], ambiguous [m]) in the channel order of the planes that
    build_sh_planes blends (the coefficients (j, rgb) flattened, then A)."""
    nc = n_coef(degree)
    pix = np.asarray(pix, dtype=np.int64).reshape(-1, 3)
    Y = np.empty((pix.shape[0], nc))
    for i, (v, y, x) in enumerate(pix):
        Y[i] = basis(pixel_directions(cam, g, float(dx32[v]), float(dy32[v]), [x], [y])[0, 0], degree)

    def colour(s):
        a = s[:, 3 * nc]
        c = np.einsum("nj,njc->nc", Y, s[:, :3 * nc].reshape(-1, nc, 3)) + 0.5 * a[:, None]
        return np.maximum(c, 0.0), a

    return composite.composite_at(texel_fn, depth32, cam, g, dx32, dy32, interp, pix, colour=colour)


def build_sh_planes(scene: dict, sh, degree: int, cam, n_chunk: int, binning="quantile", inv_depth_range=None,
                    chunks=None):
    """SH planes of a Gaussian field: (q [K,H,W,n_coef,3], A [K,H,W], ambiguous [K,H,W], depth [K]).

    The partition and the per-chunk rasterisation are those of the RGB planes; only the
    blended quantity differs (the coefficients instead of rgb)."""
    g = geometry.derive(cam)
    nc = n_coef(degree)
    part = partition.partition(scene["means"], cam, g, n_chunk, binning, inv_depth_range)
    coef = dict(scene)
    coef["rgb"] = np.asarray(sh, np.float64)[:, :nc].reshape(-1, 3 * nc)
    q = np.zeros((n_chunk, g.hp, g.wp, nc, 3))
    A = np.zeros((n_chunk, g.hp, g.wp))
    amb = np.zeros((n_chunk, g.hp, g.wp), dtype=bool)
    for k in (range(n_chunk) if chunks is None else chunks):
        proj = render.chunk_projection(coef, cam, g, part, k)
        p, amb[k] = splat.render_plane(proj, g.hp, g.wp)
        q[k] = p[..., :3 * nc].reshape(g.hp, g.wp, nc, 3)
        A[k] = p[..., 3 * nc]
    return q, A, amb, part.depth


def composite_sh(q, A, degree: int, depth32, cam, g: geometry.Geometry, dx32, dy32, interp: str = "nearest",
                 views=None) -> np.ndarray:
    """Composite SH planes into views: [nv, Ny, Nx, 4] of (Q_r, Q_g, Q_b, T).

    The texel sampling of every plane is the RGB composite's (Eq. 6 in its float32 program),
    applied to the 3 n_coef + 1 channels of the SH texels."""
    nc = n_coef(degree)
    q = np.asarray(q, np.float64)[..., :nc, :]
    K, H, W = q.shape[:3]
    stacked = np.concatenate([q.reshape(K, H, W, 3 * nc), np.asarray(A, np.float64)[..., None]], axis=-1)
    c = decisions.constants(g, cam)
    pc = decisions.plane_coeffs32(c, depth32, dx32, dy32)
    xs, ys = np.arange(g.nx), np.arange(g.ny)
    views = range(len(dx32)) if views is None else views
    outs = []
    for v in views:
        Y = basis(pixel_directions(cam, g, float(dx32[v]), float(dy32[v]), xs, ys), degree)   # [Ny, Nx, nc]
        Q = np.zeros((g.ny, g.nx, 3))
        T = np.ones((g.ny, g.nx))
        for k in range(K):
            s, _ = composite.sample_plane(stacked[k], pc, c, k, v, xs, ys, interp)             # [Ny, Nx, 3nc+1]
            qs = s[..., :3 * nc].reshape(g.ny, g.nx, nc, 3)
            a = s[..., 3 * nc]
            col = np.maximum(np.einsum("yxj,yxjc->yxc", Y, qs) + 0.5 * a[..., None], 0.0)
            Q += T[..., None] * col
            T = T * (1.0 - a)
        outs.append(np.concatenate([Q, T[..., None]], axis=-1))
    return np.stack(outs)


def render_view_sh(scene: dict, sh, degree: int, cam, dx: float = 0.0, dy: float = 0.0, dilation: float = 0.3):
    """The per-view render with SH colour: every Gaussian evaluated from view (dx, dy)."""
    coloured = dict(scene)
    coloured["rgb"] = view_colours(scene, sh, degree, cam, dx, dy)
    return render.render_view(coloured, cam, dx, dy, dilation=dilation)
