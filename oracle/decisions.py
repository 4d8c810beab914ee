"""Integer decisions taken in IEEE float32, the precision the GPU kernels take them in.

Where floating point decides an integer (is a Gaussian inside the reference
frustum, which chunk it falls into, which plane texel a view pixel samples), both
the oracle and the kernels take that decision from the same float32 values with
the same sequence of correctly rounded operations (no fused multiply-add).  Every
quantity here is an exact float32 program; the float64 geometry it approximates
lives in ``geometry`` and the two are pinned against each other in the tests.

All constants enter as float64 values rounded once to float32.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .geometry import Geometry

F = np.float32
GUARD_BAND = 1.3      # frustum guard band of the cull test (factor on tan(theta'/2))


@dataclass(frozen=True)
class Constants32:
    d_forward: np.float32
    z_near: np.float32
    guard_x: np.float32      # fl32(1.3 * tan(theta'_x/2))
    guard_y: np.float32
    ratio_x: np.float32      # fl32(f'_x / f_x): plane texels per view pixel at unit magnification
    ratio_y: np.float32
    fpx: np.float32          # fl32(f'_x)
    fpy: np.float32
    cpx: np.float32          # (W_p - 1)/2, exact
    cpy: np.float32
    cx: np.float32           # (N_x - 1)/2, exact
    cy: np.float32
    inv_focal: np.float32    # fl32(1 / D_focal)


def constants(g: Geometry, cam) -> Constants32:
    return Constants32(
        d_forward=F(g.d_forward), z_near=F(cam.z_near),
        guard_x=F(GUARD_BAND * g.tpx), guard_y=F(GUARD_BAND * g.tpy),
        ratio_x=F((g.wp * g.tx) / (g.nx * g.tpx)), ratio_y=F((g.hp * g.ty) / (g.ny * g.tpy)),
        fpx=F(g.fpx), fpy=F(g.fpy), cpx=F(g.cpx), cpy=F(g.cpy), cx=F(g.cx), cy=F(g.cy),
        inv_focal=F(1.0 / g.d_focal))


def camera_coords32(points32: np.ndarray, cam):
    """Base-camera coordinates in float32: c_r = ((R[r,0] x + R[r,1] y) + R[r,2] z) + t[r]."""
    R = np.asarray(cam.R, dtype=np.float32).reshape(3, 3)
    t = np.asarray(cam.t, dtype=np.float32)
    x, y, z = (np.ascontiguousarray(points32[:, i], dtype=np.float32) for i in range(3))

    def row(r):
        return ((R[r, 0] * x + R[r, 1] * y) + R[r, 2] * z) + t[r]
    with np.errstate(invalid="ignore", over="ignore"):
        return row(0), row(1), row(2)


def keys_and_cull(points32: np.ndarray, cam, c: Constants32):
    """Depth key (base-camera z) and reference-frustum visibility, both in float32.

    A primitive is visible iff its key and lateral coordinates are finite and
    z_ref = fl(key - D_forward) > z_near, |x_c| <= fl(guard_x * z_ref), |y_c| <= fl(guard_y * z_ref).
    A negative zero key is replaced by +0 so that equal keys compare equal bitwise.
    """
    xc, yc, key = camera_coords32(points32, cam)
    key = key + F(0.0)
    with np.errstate(invalid="ignore", over="ignore"):
        zr = key - c.d_forward
        vis = (np.isfinite(key) & np.isfinite(xc) & np.isfinite(yc) & (zr > c.z_near)
               & (np.abs(xc) <= c.guard_x * zr) & (np.abs(yc) <= c.guard_y * zr))
    return key.astype(np.float32), vis


def inv_depth_edges32(n_chunk: int, z_lo: float, z_hi: float) -> np.ndarray:
    """Interior edges E_1..E_{K-1} of K planes uniform in inverse depth, rounded to float32.

    1/E_i = 1/z_lo + (i/K)(1/z_hi - 1/z_lo), evaluated in float64.
    """
    i = np.arange(1, n_chunk, dtype=np.float64)
    inv = 1.0 / z_lo + (i / n_chunk) * (1.0 / z_hi - 1.0 / z_lo)
    return (1.0 / inv).astype(np.float32)


@dataclass(frozen=True)
class PlaneCoeffs32:
    """Per-plane slope and per-(plane, view) offset of the texel coordinate, float32.

    For view pixel (x, y) the texel coordinate on plane k in view v is
        X = fl(fl(bx[k] * fl(x - cx)) + Cx[k, v]),  Y likewise,
    where ``Cx`` holds the bilinear offsets and ``Cxn = fl(Cx + 1/2)`` the offsets whose
    floor is the nearest texel.  In exact arithmetic X equals Eq. 6 mapped to texels:
        X = c'_x + (f'_x/f_x) d/(d - D_fwd) (x - c_x) + f'_x dx (1 - d/D_focal)/(d - D_fwd).
    """
    bx: np.ndarray
    by: np.ndarray
    Cx: np.ndarray
    Cy: np.ndarray
    Cxn: np.ndarray
    Cyn: np.ndarray


def plane_coeffs32(c: Constants32, depth32: np.ndarray, dx32: np.ndarray, dy32: np.ndarray) -> PlaneCoeffs32:
    d = np.asarray(depth32, dtype=np.float32)
    z = d - c.d_forward
    q = d / z
    w = (F(1.0) - d * c.inv_focal) / z
    bx = c.ratio_x * q
    by = c.ratio_y * q
    gx = c.fpx * w
    gy = c.fpy * w
    dx = np.asarray(dx32, dtype=np.float32)
    dy = np.asarray(dy32, dtype=np.float32)
    Cx = c.cpx + gx[:, None] * dx[None, :]
    Cy = c.cpy + gy[:, None] * dy[None, :]
    return PlaneCoeffs32(bx=bx, by=by, Cx=Cx, Cy=Cy, Cxn=Cx + F(0.5), Cyn=Cy + F(0.5))


def texel_coords32(pc: PlaneCoeffs32, c: Constants32, k: int, v: int, xs, ys, nearest: bool):
    """Float32 texel coordinates (X over ``xs``, Y over ``ys``) of plane k in view v."""
    xr = np.asarray(xs, dtype=np.float32) - c.cx
    yr = np.asarray(ys, dtype=np.float32) - c.cy
    Cx = pc.Cxn[k, v] if nearest else pc.Cx[k, v]
    Cy = pc.Cyn[k, v] if nearest else pc.Cy[k, v]
    X = pc.bx[k] * xr + Cx
    Y = pc.by[k] * yr + Cy
    return X.astype(np.float32), Y.astype(np.float32)
