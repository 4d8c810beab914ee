"""Rasterise each chunk into its sweeping plane, float64 (Alg. 1 "Rasterize"; Sec. 4.4).

For chunk k and texel centre p, over the chunk's Gaussians in (depth key, index)
order, starting from T = 1 and C = 0:

    a = o G(p);  if a >= 1/255:  alpha = min(0.99, a);  C += alpha T rgb;  T *= 1 - alpha

with no early termination.  The plane stores premultiplied RGBA (C, 1 - T): the
colour is already weighted by opacity, as Eq. 7 requires of the sampled c_k, and
the alpha channel is one minus the chunk's transmittance.

Ambiguity.  The inclusion rule a >= 1/255 is a threshold on a float value; a kernel
computing G in float32 may decide differently from this float64 code when a lies
within its rounding error of 1/255, and both outcomes are then correct.  Each texel
records whether any of its Gaussians satisfies |ln(a) - ln(1/255)| <= eps_g, with
eps_g = AMBIGUITY_BASE * (1 + cond(Sigma')), a float32 error bound of ln G (the
quadratic form loses accuracy in proportion to the conditioning of Sigma').
"""
from __future__ import annotations

import math

import numpy as np

from .project import ALPHA_MAX, ALPHA_MIN, Projected

AMBIGUITY_BASE = 4e-6
LN_ALPHA_MIN = math.log(ALPHA_MIN)


def ambiguity_eps(cov2d: np.ndarray) -> np.ndarray:
    ev = np.linalg.eigvalsh(cov2d)
    return AMBIGUITY_BASE * (1.0 + ev[..., 1] / ev[..., 0])


def support_halfwidth(proj: Projected, eps: np.ndarray):
    """Half-widths of the bounding box of {p : ln(o G(p)) >= ln(1/255) - eps}."""
    r2 = 2.0 * (np.log(proj.opacity) - LN_ALPHA_MIN + eps)
    r2 = np.where(np.isfinite(r2), r2, -1.0)
    ok = r2 >= 0.0
    r2 = np.maximum(r2, 0.0)
    return np.sqrt(r2 * proj.cov2d[:, 0, 0]), np.sqrt(r2 * proj.cov2d[:, 1, 1]), ok


def render_plane(proj: Projected, height: int, width: int, eps=None):
    """One plane from the Gaussians of one chunk, given in front-to-back order.

    Returns (rgba [H,W,4] float64, ambiguous [H,W] bool).  The colour may have any number
    of channels c (proj.rgb [n,c]; the planes of spherical-harmonic coefficients blend the
    coefficients the same way), and the result then has c + 1 channels, alpha last.
    """
    C = np.zeros((height, width, proj.rgb.shape[1]))
    T = np.ones((height, width))
    amb = np.zeros((height, width), dtype=bool)
    n = proj.mean2d.shape[0]
    if n == 0:
        return np.concatenate([C, (1.0 - T)[..., None]], axis=-1), amb
    if eps is None:
        eps = ambiguity_eps(proj.cov2d)
    hx, hy, ok = support_halfwidth(proj, eps)
    for i in range(n):
        if not ok[i]:
            continue
        mx, my = proj.mean2d[i]
        x0, x1 = max(0, math.ceil(mx - hx[i])), min(width - 1, math.floor(mx + hx[i]))
        y0, y1 = max(0, math.ceil(my - hy[i])), min(height - 1, math.floor(my + hy[i]))
        if x0 > x1 or y0 > y1:
            continue
        xs = np.arange(x0, x1 + 1, dtype=np.float64) - mx
        ys = np.arange(y0, y1 + 1, dtype=np.float64) - my
        dx = xs[None, :]
        dy = ys[:, None]
        Q = proj.conic[i]
        quad = Q[0, 0] * dx * dx + (Q[0, 1] + Q[1, 0]) * dx * dy + Q[1, 1] * dy * dy
        ln_a = math.log(proj.opacity[i]) - 0.5 * quad
        inc = ln_a >= LN_ALPHA_MIN
        alpha = np.where(inc, np.minimum(ALPHA_MAX, np.exp(ln_a)), 0.0)
        sl = (slice(y0, y1 + 1), slice(x0, x1 + 1))
        Tr = T[sl]
        C[sl] += (alpha * Tr)[..., None] * proj.rgb[i]
        T[sl] = Tr * (1.0 - alpha)
        amb[sl] |= np.abs(ln_a - LN_ALPHA_MIN) <= eps[i]
    return np.concatenate([C, (1.0 - T)[..., None]], axis=-1), amb


def blend_texels(proj: Projected, px: np.ndarray, py: np.ndarray, eps=None):
    """Premultiplied RGBA of one chunk at arbitrary texel positions (vectorised over Gaussians).

    Returns (rgba [n,4], ambiguous [n]); with c colour channels, [n, c + 1] (alpha last).
    """
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    nc = proj.rgb.shape[1]
    out = np.zeros((px.size, nc + 1))
    amb = np.zeros(px.size, dtype=bool)
    ng = proj.mean2d.shape[0]
    if ng == 0:
        return out, amb
    if eps is None:
        eps = ambiguity_eps(proj.cov2d)
    lno = np.log(proj.opacity)
    step = max(1, 4_000_000 // max(ng, 1))
    for s in range(0, px.size, step):
        dx = px[s:s + step][None, :] - proj.mean2d[:, 0:1]
        dy = py[s:s + step][None, :] - proj.mean2d[:, 1:2]
        Q = proj.conic
        quad = (Q[:, 0, 0:1] * dx * dx + (Q[:, 0, 1:2] + Q[:, 1, 0:1]) * dx * dy
                + Q[:, 1, 1:2] * dy * dy)
        ln_a = lno[:, None] - 0.5 * quad
        inc = ln_a >= LN_ALPHA_MIN
        alpha = np.where(inc, np.minimum(ALPHA_MAX, np.exp(np.minimum(ln_a, 0.0))), 0.0)
        Tin = np.cumprod(np.concatenate([np.ones((1, alpha.shape[1])), 1.0 - alpha[:-1]], axis=0), axis=0)
        w = alpha * Tin
        out[s:s + step, :nc] = w.T @ proj.rgb
        out[s:s + step, nc] = 1.0 - Tin[-1] * (1.0 - alpha[-1])
        amb[s:s + step] = np.any(np.abs(ln_a - LN_ALPHA_MIN) <= eps[:, None], axis=0)
    return out, amb


def support_pairs(proj: Projected, height: int, width: int, eps=None):
    """The support pairs of one chunk: the number of (Gaussian, texel) pairs of the
    height x width plane with o G >= 1/255 (the texels the blend above gives a non-zero
    alpha), and the number of those pairs within eps_g of the threshold, where a float32
    decision may go either way (both returned as ints)."""
    n = proj.mean2d.shape[0]
    if n == 0:
        return 0, 0
    if eps is None:
        eps = ambiguity_eps(proj.cov2d)
    hx, hy, ok = support_halfwidth(proj, eps)
    inside, near = 0, 0
    for i in range(n):
        if not ok[i]:
            continue
        mx, my = proj.mean2d[i]
        x0, x1 = max(0, math.ceil(mx - hx[i])), min(width - 1, math.floor(mx + hx[i]))
        y0, y1 = max(0, math.ceil(my - hy[i])), min(height - 1, math.floor(my + hy[i]))
        if x0 > x1 or y0 > y1:
            continue
        dx = (np.arange(x0, x1 + 1, dtype=np.float64) - mx)[None, :]
        dy = (np.arange(y0, y1 + 1, dtype=np.float64) - my)[:, None]
        Q = proj.conic[i]
        quad = Q[0, 0] * dx * dx + (Q[0, 1] + Q[1, 0]) * dx * dy + Q[1, 1] * dy * dy
        ln_a = math.log(proj.opacity[i]) - 0.5 * quad
        inside += int((ln_a >= LN_ALPHA_MIN).sum())
        near += int((np.abs(ln_a - LN_ALPHA_MIN) <= eps[i]).sum())
    return inside, near
