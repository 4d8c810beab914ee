"""Display geometry in float64 (Sec. 4.2 "Sweeping planes rendering", Sec. 4.3 "Swizzle blending").

Conventions (the paper is silent on them): the base camera looks along +z with x
to the right and y down; pixel x of an N-pixel row has its centre at NDC
u = (2x+1)/N - 1, so texel centres sit at integer pixel coordinates and NDC +-1 at
the outer edges; all angles are full angles.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def round_half_up(v: float) -> int:
    return int(math.floor(v + 0.5))


@dataclass(frozen=True)
class Geometry:
    d_focal: float
    tx: float            # tan(theta_x / 2) of the base camera
    ty: float
    taux: float          # tan(phi_x / 2) of the display viewing angle
    tauy: float
    d_forward0: float    # Eq. 1, before the D_shift adjustment
    d_forward: float     # reference camera position on the base camera's z axis
    tpx: float           # tan(theta'_x / 2), Eq. 2
    tpy: float
    nx: int
    ny: int
    wp: int              # plane resolution = round(P_s * N)
    hp: int
    fx: float            # base (view) focal length in pixels
    fy: float
    cx: float            # base principal point (pixel units)
    cy: float
    fpx: float           # reference focal length in plane texels
    fpy: float
    cpx: float
    cpy: float
    f_dilation: float    # Eq. 8, in reference texels^2
    plane_scale: float


def derive(cam) -> Geometry:
    """Reference camera and plane geometry for a display setup.

    Eq. 1: D_forward = max_k D_focal * tan(phi_k/2) / (tan(phi_k/2) + tan(theta_k/2)).
    Eq. 2: tan(theta'_k/2) = D_focal * tan(theta_k/2) / (D_focal - D_forward).
    D_shift moves the reference camera back after theta' is fixed (Sec. 4.2); theta'
    uses the unshifted D_forward.
    Eq. 8: f' = 0.3 * (D_focal tan(theta_x/2) / ((D_focal - D_forward) tan(theta'_x/2)) * P_s)^2,
    unless the camera sets a positive constant ``dilation`` (the constant filter of the
    adaptive-filter ablation, Sec. 5).
    """
    Df = float(cam.d_focal)
    tx, ty = math.tan(0.5 * cam.fov_x), math.tan(0.5 * cam.fov_y)
    taux, tauy = math.tan(0.5 * cam.phi_x), math.tan(0.5 * cam.phi_y)
    d0 = max(Df * taux / (taux + tx), Df * tauy / (tauy + ty))
    tpx = Df * tx / (Df - d0)
    tpy = Df * ty / (Df - d0)
    dfwd = d0 - float(cam.d_shift)
    ps = float(cam.plane_scale)
    wp, hp = round_half_up(ps * cam.nx), round_half_up(ps * cam.ny)
    const = float(getattr(cam, "dilation", 0.0))
    fdil = const if const > 0.0 else 0.3 * (Df * tx / ((Df - dfwd) * tpx) * ps) ** 2
    return Geometry(d_focal=Df, tx=tx, ty=ty, taux=taux, tauy=tauy, d_forward0=d0, d_forward=dfwd,
                    tpx=tpx, tpy=tpy, nx=int(cam.nx), ny=int(cam.ny), wp=wp, hp=hp,
                    fx=0.5 * cam.nx / tx, fy=0.5 * cam.ny / ty, cx=0.5 * (cam.nx - 1), cy=0.5 * (cam.ny - 1),
                    fpx=0.5 * wp / tpx, fpy=0.5 * hp / tpy, cpx=0.5 * (wp - 1), cpy=0.5 * (hp - 1),
                    f_dilation=fdil, plane_scale=ps)


def view_positions(n: int) -> np.ndarray:
    """Eq. 3: s_j = (j-1)/(V-1) - 1/2 for j = 1..V; a single view sits at s = 0."""
    if n == 1:
        return np.zeros(1)
    return np.arange(n, dtype=np.float64) / (n - 1) - 0.5


def quilt_views(cam, vx: int, vy: int):
    """Lateral offsets (Eq. 4) and normalised principal-point shifts (Eq. 5) of the quilt.

    Views are ordered row-major: index = i * vx + j (row i over vy, column j over vx).
    Returns float64 arrays dx, dy, px, py of length vx*vy.
    """
    g = derive(cam)
    sx, sy = view_positions(vx), view_positions(vy)
    dxj = 2.0 * g.d_focal * sx * g.taux
    dyi = 2.0 * g.d_focal * sy * g.tauy
    pxj = 2.0 * sx * g.taux / g.tx
    pyi = 2.0 * sy * g.tauy / g.ty
    dx = np.tile(dxj, vy)
    px = np.tile(pxj, vy)
    dy = np.repeat(dyi, vx)
    py = np.repeat(pyi, vx)
    return dx, dy, px, py


def u_prime(g: Geometry, dx, d, u):
    """Eq. 6: NDC coordinate on the plane at base depth d of view pixel NDC u, view offset dx."""
    return (dx * (g.d_focal - d) / g.d_focal + d * g.tx * u) / ((d - g.d_forward) * g.tpx)


def v_prime(g: Geometry, dy, d, v):
    """Vertical counterpart of Eq. 6."""
    return (dy * (g.d_focal - d) / g.d_focal + d * g.ty * v) / ((d - g.d_forward) * g.tpy)


def pixel_ndc(x, n):
    return (2.0 * np.asarray(x, dtype=np.float64) + 1.0) / n - 1.0


def ndc_to_texel(up, n):
    return (np.asarray(up, dtype=np.float64) + 1.0) * n / 2.0 - 0.5
