"""Swizzle blending of sweeping planes into light-field views (Sec. 4.3, Eqs. 6-7, Alg. 1).

For view v with lateral offset (dx, dy) and pixel (x, y), planes are visited front
to back (k = 0..K-1).  Each plane is sampled at the texel coordinate of Eq. 6 and
the samples are over-composited (Eq. 7; the colours are premultiplied):

    Q = 0, T = 1;  for k:  (c, a) = sample_k(X, Y);  Q += T c;  T *= 1 - a.

Sampling a premultiplied RGBA plane is linear, so interpolating (C, A = 1 - T_k)
equals interpolating C and T separately as Alg. 1 does.  Texels outside the plane
are transparent (0, 0, 0, 0) - that region is the near field excluded from the
reference frustum (Sec. 4.2).  Nearest sampling takes the texel floor(X + 1/2);
bilinear takes the four texels around (X, Y) with the usual weights.  The texel
coordinates are the float32 program of ``decisions.plane_coeffs32`` (see there);
the blending itself runs in float64.

Output per pixel: (Q_r, Q_g, Q_b, T) - Alg. 1 returns the quilt Q and the
transmittance buffer T; no background is added.
"""
from __future__ import annotations

import numpy as np

from . import decisions


def _sample_rows_cols(plane, iy, ix):
    """plane[iy][:, ix] with zeros outside; iy, ix int arrays (any values)."""
    H, W = plane.shape[:2]
    vy = (iy >= 0) & (iy < H)
    vx = (ix >= 0) & (ix < W)
    s = plane[np.clip(iy, 0, H - 1)][:, np.clip(ix, 0, W - 1)]
    return s * (vy[:, None] & vx[None, :])[..., None]


def _sample_mask(mask, iy, ix):
    H, W = mask.shape
    vy = (iy >= 0) & (iy < H)
    vx = (ix >= 0) & (ix < W)
    return mask[np.clip(iy, 0, H - 1)][:, np.clip(ix, 0, W - 1)] & (vy[:, None] & vx[None, :])


def sample_plane(plane, pc, c, k: int, v: int, xs, ys, interp: str, mask=None):
    """Plane k [H,W,C] sampled at the pixels (xs x ys) of view v (Eq. 6): returns (s [Ny,Nx,C],
    whether a sample touches a masked texel [Ny,Nx] or None without a mask)."""
    if interp == "nearest":
        X, Y = decisions.texel_coords32(pc, c, k, v, xs, ys, nearest=True)
        ix = np.floor(X).astype(np.int64)
        iy = np.floor(Y).astype(np.int64)
        s = _sample_rows_cols(plane, iy, ix)
        return s, (None if mask is None else _sample_mask(mask, iy, ix))
    if interp != "bilinear":
        raise ValueError(interp)
    X, Y = decisions.texel_coords32(pc, c, k, v, xs, ys, nearest=False)
    x0 = np.floor(X)
    y0 = np.floor(Y)
    wx = X.astype(np.float64) - x0
    wy = Y.astype(np.float64) - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    s = 0.0
    pa = None if mask is None else np.zeros((len(ys), len(xs)), dtype=bool)
    for oy, fy in ((0, 1.0 - wy), (1, wy)):
        for ox, fx in ((0, 1.0 - wx), (1, wx)):
            wgt = fy[:, None] * fx[None, :]
            s = s + _sample_rows_cols(plane, y0 + oy, x0 + ox) * wgt[..., None]
            if mask is not None:
                pa |= _sample_mask(mask, y0 + oy, x0 + ox) & (wgt > 0)
    return s, pa


def composite(planes, depth32, cam, geom, dx32, dy32, interp: str = "nearest", amb=None, views=None):
    """Composite all pixels of the selected views.

    planes [K,H,W,4] premultiplied RGBA (any float dtype, used as float64); depth32 [K]
    float32 plane depths; dx32, dy32 float32 view offsets.  Returns (out [nv,Ny,Nx,4] float64,
    ambiguous [nv,Ny,Nx] bool) - a pixel is ambiguous when it samples an ambiguous texel.
    """
    planes = np.asarray(planes, dtype=np.float64)
    K = planes.shape[0]
    c = decisions.constants(geom, cam)
    pc = decisions.plane_coeffs32(c, depth32, dx32, dy32)
    views = range(len(dx32)) if views is None else views
    Nx, Ny = geom.nx, geom.ny
    xs, ys = np.arange(Nx), np.arange(Ny)
    outs, ambs = [], []
    for v in views:
        Q = np.zeros((Ny, Nx, 3))
        T = np.ones((Ny, Nx))
        pa = np.zeros((Ny, Nx), dtype=bool)
        for k in range(K):
            s, m = sample_plane(planes[k], pc, c, k, v, xs, ys, interp, None if amb is None else amb[k])
            if m is not None:
                pa |= m
            Q += T[..., None] * s[..., :3]
            T = T * (1.0 - s[..., 3])
        outs.append(np.concatenate([Q, T[..., None]], axis=-1))
        ambs.append(pa)
    return np.stack(outs), np.stack(ambs)


def composite_at(texel_fn, depth32, cam, geom, dx32, dy32, interp: str, pix, colour=None):
    """Composite individual pixels; ``pix`` is an int array [n,3] of (view, y, x).

    ``texel_fn(k, iy, ix)`` returns (rgba [m,4], ambiguous [m]) of plane k at in-range
    integer texels.  Returns (out [n,4], ambiguous [n]).  For texels of other channels,
    ``colour(s)`` maps the samples s [n, C] to (premultiplied colour [n,3], alpha [n]).
    """
    pix = np.asarray(pix, dtype=np.int64).reshape(-1, 3)
    K = len(depth32)
    c = decisions.constants(geom, cam)
    pc = decisions.plane_coeffs32(c, depth32, dx32, dy32)
    n = pix.shape[0]
    Q = np.zeros((n, 3))
    T = np.ones(n)
    pa = np.zeros(n, dtype=bool)
    W, H = geom.wp, geom.hp
    nearest = interp == "nearest"
    by_view = np.argsort(pix[:, 0], kind="stable")          # the pixels of each view, found once
    views, starts = np.unique(pix[by_view, 0], return_index=True)
    groups = [(int(v), by_view[s:e]) for v, s, e in zip(views, starts, list(starts[1:]) + [n])]
    for k in range(K):
        X = np.empty(n, dtype=np.float32)
        Y = np.empty(n, dtype=np.float32)
        for v, sel in groups:
            X[sel], Y[sel] = decisions.texel_coords32(pc, c, k, v, pix[sel, 2], pix[sel, 1], nearest)
        if nearest:
            taps = [(np.floor(Y).astype(np.int64), np.floor(X).astype(np.int64), np.ones(n))]
        else:
            x0 = np.floor(X)
            y0 = np.floor(Y)
            wx = X.astype(np.float64) - x0
            wy = Y.astype(np.float64) - y0
            x0 = x0.astype(np.int64)
            y0 = y0.astype(np.int64)
            taps = [(y0 + oy, x0 + ox, fy * fx) for oy, fy in ((0, 1 - wy), (1, wy))
                    for ox, fx in ((0, 1 - wx), (1, wx))]
        s = None
        for iy, ix, w in taps:
            ok = (iy >= 0) & (iy < H) & (ix >= 0) & (ix < W)
            val, am = texel_fn(k, iy[ok], ix[ok])
            if s is None:
                s = np.zeros((n, val.shape[1]))
            if np.any(ok):
                s[ok] += val * w[ok, None]
                pa[np.nonzero(ok)[0][am & (w[ok] > 0)]] = True
        col, alpha = (s[:, :3], s[:, 3]) if colour is None else colour(s)
        Q += T[:, None] * col
        T = T * (1.0 - alpha)
    return np.concatenate([Q, T[:, None]], axis=1), pa
