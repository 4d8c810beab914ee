"""Gradients of a multi-view L2 loss through the whole light-field pipeline (test
infrastructure; torch CPU float64 autograd).

The forward is the oracle's own pipeline restated in torch: EWA projection into the
reference camera (``project``), front-to-back rasterisation of each chunk into a
premultiplied plane (``splat``), and the swizzle composite of the views (``composite``),
with loss L = sum over views, pixels and RGB of (Q - Q*)^2.  Every discrete decision is
taken once, at the parameters the gradient is evaluated at, and then held fixed (the
gradient is that of the smooth piece containing those parameters):

* the partition (chunk of every Gaussian, plane depths d_k: stop-gradient),
* which (Gaussian, texel) pairs are included (o G >= 1/255) and which are clamped to 0.99,
* the composite's texel indices (nearest) and bilinear weights, taken by the float32
  coordinate program of ``decisions``.

``frozen_loss`` evaluates the loss at other parameters with the same decisions, which is
what central finite differences need.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import composite, decisions, geometry, partition, project, splat

KEYS = ("means", "log_scales", "quats", "opacity", "rgb")
TD = torch.float64


@dataclass
class Decisions:
    geom: geometry.Geometry
    part: partition.Partition
    # included (Gaussian, texel) pairs, sorted by (plane, texel, rank)
    gauss: np.ndarray        # [P] Gaussian index
    plane: np.ndarray        # [P] chunk k
    texel: np.ndarray        # [P] flat texel index y * W + x within the plane
    clamped: np.ndarray      # [P] bool: alpha = 0.99
    group: np.ndarray        # [P] id of the (plane, texel) group
    group_start: np.ndarray  # [G] first pair of each group
    group_cell: np.ndarray   # [G] flat (k, texel) index of each group
    # composite taps: for each plane, flat texel index and weight per (view, pixel, tap)
    taps_idx: list           # K arrays [V*Ny*Nx, ntap] int64 (-1: outside the plane)
    taps_w: list             # K arrays [V*Ny*Nx, ntap] float64
    n_views: int


def _pairs(scene, cam, g, part, K):
    gs, ks, ts, cl = [], [], [], []
    for k in range(K):
        idx = part.order[part.chunk_start[k]:part.chunk_start[k + 1]]
        if idx.size == 0:
            continue
        pr = project.project_reference(scene, idx, cam, g)
        hx, hy, ok = splat.support_halfwidth(pr, np.zeros(idx.size))
        for r, i in enumerate(idx):
            if not ok[r]:
                continue
            mx, my = pr.mean2d[r]
            x0, x1 = max(0, math.ceil(mx - hx[r])), min(g.wp - 1, math.floor(mx + hx[r]))
            y0, y1 = max(0, math.ceil(my - hy[r])), min(g.hp - 1, math.floor(my + hy[r]))
            if x0 > x1 or y0 > y1:
                continue
            yy, xx = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
            dx, dy = xx - mx, yy - my
            Q = pr.conic[r]
            ln_a = math.log(pr.opacity[r]) - 0.5 * (Q[0, 0] * dx * dx + (Q[0, 1] + Q[1, 0]) * dx * dy + Q[1, 1] * dy * dy)
            inc = ln_a >= splat.LN_ALPHA_MIN
            n = int(inc.sum())
            if n == 0:
                continue
            gs.append(np.full(n, i))
            ks.append(np.full(n, k))
            ts.append((yy * g.wp + xx)[inc])
            cl.append((np.exp(ln_a) >= project.ALPHA_MAX)[inc])
    if not gs:
        z = np.zeros(0, dtype=np.int64)
        return z, z, z, np.zeros(0, dtype=bool)
    return np.concatenate(gs), np.concatenate(ks), np.concatenate(ts), np.concatenate(cl)


def decide(scene: dict, cam, n_chunk: int, dx32, dy32, interp: str = "nearest", binning="quantile",
           inv_depth_range=None) -> Decisions:
    """Take every discrete decision of the forward at the scene's parameters."""
    g = geometry.derive(cam)
    part = partition.partition(scene["means"], cam, g, n_chunk, binning, inv_depth_range)
    gauss, plane, texel, clamped = _pairs(scene, cam, g, part, n_chunk)
    # pairs arrive per plane in rank order; a stable sort by (plane, texel) keeps rank order
    order = np.lexsort((texel, plane))
    gauss, plane, texel, clamped = gauss[order], plane[order], texel[order], clamped[order]
    cell = plane.astype(np.int64) * (g.hp * g.wp) + texel
    new = np.ones(cell.size, dtype=bool)
    new[1:] = cell[1:] != cell[:-1]
    group = np.cumsum(new) - 1
    group_start = np.nonzero(new)[0]
    taps_idx, taps_w = composite_taps(cam, g, part.depth, dx32, dy32, interp)
    return Decisions(geom=g, part=part, gauss=gauss, plane=plane, texel=texel, clamped=clamped, group=group,
                     group_start=group_start, group_cell=cell[group_start], taps_idx=taps_idx, taps_w=taps_w,
                     n_views=len(dx32))


def composite_taps(cam, g: geometry.Geometry, depth32, dx32, dy32, interp: str):
    """Per plane: texel indices [V*Ny*Nx, ntap] (-1 outside the plane) and weights of every
    view pixel's sample, from the float32 coordinate program (nearest: 1 tap, bilinear: 4)."""
    c = decisions.constants(g, cam)
    pc = decisions.plane_coeffs32(c, np.asarray(depth32, np.float32), np.asarray(dx32, np.float32),
                                  np.asarray(dy32, np.float32))
    V = len(dx32)
    ys, xs = np.meshgrid(np.arange(cam.ny), np.arange(cam.nx), indexing="ij")
    xs, ys = xs.reshape(-1), ys.reshape(-1)
    taps_idx, taps_w = [], []
    nearest = interp == "nearest"
    for k in range(len(depth32)):
        ii, ww = [], []
        for v in range(V):
            X, Y = decisions.texel_coords32(pc, c, k, v, xs, ys, nearest)
            if nearest:
                taps = [(np.floor(Y).astype(np.int64), np.floor(X).astype(np.int64), np.ones(xs.size))]
            else:
                x0, y0 = np.floor(X), np.floor(Y)
                wx, wy = X.astype(np.float64) - x0, Y.astype(np.float64) - y0
                x0, y0 = x0.astype(np.int64), y0.astype(np.int64)
                taps = [(y0 + oy, x0 + ox, fy * fx) for oy, fy in ((0, 1 - wy), (1, wy)) for ox, fx in ((0, 1 - wx), (1, wx))]
            idx = np.stack([np.where((iy >= 0) & (iy < g.hp) & (ix >= 0) & (ix < g.wp), iy * g.wp + ix, -1)
                            for iy, ix, _ in taps], axis=1)
            ii.append(idx)
            ww.append(np.stack([w for _, _, w in taps], axis=1))
        taps_idx.append(np.concatenate(ii))
        taps_w.append(np.concatenate(ww))
    return taps_idx, taps_w


@dataclass
class CompositeTaps:
    geom: geometry.Geometry
    taps_idx: list
    taps_w: list
    n_views: int


def composite_decisions(cam, depth32, dx32, dy32, interp: str = "nearest") -> CompositeTaps:
    """The composite's frozen sampling for given plane depths (no scene needed)."""
    g = geometry.derive(cam)
    ti, tw = composite_taps(cam, g, depth32, dx32, dy32, interp)
    return CompositeTaps(geom=g, taps_idx=ti, taps_w=tw, n_views=len(dx32))


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def project_reference(p: dict, cam, g: geometry.Geometry):
    """Projected means [N,2] and inverse 2D covariances [N,2,2] (EWA, Eq. 8 dilation)."""
    Rc = torch.tensor(np.asarray(cam.R, np.float64).reshape(3, 3), dtype=TD)
    tc = torch.tensor(np.asarray(cam.t, np.float64), dtype=TD)
    pc = p["means"] @ Rc.T + tc
    x, y, z = pc[:, 0], pc[:, 1], pc[:, 2] - g.d_forward
    mean2d = torch.stack([g.fpx * x / z + g.cpx, g.fpy * y / z + g.cpy], -1)
    R = quat_to_rot(p["quats"])
    sig = R @ torch.diag_embed(torch.exp(2.0 * p["log_scales"])) @ R.transpose(-1, -2)
    sig_c = Rc @ sig @ Rc.T
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([g.fpx / z, zero, -g.fpx * x / (z * z)], -1),
                     torch.stack([zero, g.fpy / z, -g.fpy * y / (z * z)], -1)], -2)
    cov = J @ sig_c @ J.transpose(-1, -2) + g.f_dilation * torch.eye(2, dtype=TD)
    return mean2d, torch.linalg.inv(cov)


def planes_of(p: dict, cam, d: Decisions, n_chunk: int) -> torch.Tensor:
    """Premultiplied planes [K, H, W, 4] (C, 1 - T) from the frozen pair list."""
    g = d.geom
    mean2d, conic = project_reference(p, cam, g)
    gi = torch.from_numpy(d.gauss)
    px = torch.from_numpy((d.texel % g.wp).astype(np.float64))
    py = torch.from_numpy((d.texel // g.wp).astype(np.float64))
    dx, dy = px - mean2d[gi, 0], py - mean2d[gi, 1]
    Q = conic[gi]
    quad = Q[:, 0, 0] * dx * dx + (Q[:, 0, 1] + Q[:, 1, 0]) * dx * dy + Q[:, 1, 1] * dy * dy
    a = p["opacity"][gi] * torch.exp(-0.5 * quad)
    alpha = torch.where(torch.from_numpy(d.clamped), torch.full_like(a, project.ALPHA_MAX), a)
    log1m = torch.log1p(-alpha)
    cs = torch.cumsum(log1m, 0)
    before = cs - log1m                                      # inclusive sum of the earlier pairs
    start = torch.from_numpy(d.group_start)
    base = before[start][torch.from_numpy(d.group)]
    T = torch.exp(before - base)                             # transmittance in front of the pair
    ncell = n_chunk * g.hp * g.wp
    cells = torch.from_numpy(d.plane.astype(np.int64) * (g.hp * g.wp) + d.texel)
    C = torch.zeros(ncell, 3, dtype=TD).index_add(0, cells, (T * alpha)[:, None] * p["rgb"][gi])
    tot = torch.zeros(ncell, dtype=TD).index_add(0, cells, log1m)
    A = 1.0 - torch.exp(tot)
    return torch.cat([C, A[:, None]], 1).reshape(n_chunk, g.hp, g.wp, 4)


def composite_of(planes: torch.Tensor, d: Decisions, cam) -> torch.Tensor:
    """Views [V, Ny, Nx, 4] = (Q, T) of planes [K, H, W, 4] through the frozen taps."""
    K = planes.shape[0]
    n = d.n_views * cam.ny * cam.nx
    Q = torch.zeros(n, 3, dtype=planes.dtype)
    T = torch.ones(n, dtype=planes.dtype)
    for k in range(K):
        flat = planes[k].reshape(-1, 4)
        idx = torch.from_numpy(d.taps_idx[k])
        w = torch.from_numpy(d.taps_w[k]) * (idx >= 0)
        s = (flat[idx.clamp(min=0)] * w[..., None]).sum(1)
        Q = Q + T[:, None] * s[:, :3]
        T = T * (1.0 - s[:, 3])
    return torch.cat([Q, T[:, None]], 1).reshape(d.n_views, cam.ny, cam.nx, 4)


def params_of(scene: dict, requires_grad: bool = True) -> dict:
    return {k: torch.tensor(np.asarray(scene[k], np.float64), dtype=TD, requires_grad=requires_grad) for k in KEYS}


def frozen_loss(p: dict, cam, d: Decisions, n_chunk: int, target: torch.Tensor):
    """L = sum (Q - Q*)^2 over views, pixels and RGB, with the decisions ``d``."""
    views = composite_of(planes_of(p, cam, d, n_chunk), d, cam)
    return ((views[..., :3] - target[..., :3]) ** 2).sum(), views


def loss_and_grad(scene: dict, cam, n_chunk: int, dx32, dy32, target, interp="nearest", d: Decisions = None):
    """Loss, views and the gradient w.r.t. every Gaussian parameter (dict of numpy arrays)."""
    if d is None:
        d = decide(scene, cam, n_chunk, dx32, dy32, interp)
    p = params_of(scene)
    tgt = torch.as_tensor(np.asarray(target, np.float64))
    loss, views = frozen_loss(p, cam, d, n_chunk, tgt)
    loss.backward()
    return float(loss.detach()), views.detach().numpy(), {k: p[k].grad.numpy() for k in KEYS}, d


def planes_vjp(scene: dict, cam, n_chunk: int, d: Decisions, d_planes: np.ndarray) -> dict:
    """Gradient w.r.t. the Gaussian parameters of <d_planes, planes(params)> (the build's VJP)."""
    p = params_of(scene)
    planes = planes_of(p, cam, d, n_chunk)
    (planes * torch.as_tensor(d_planes, dtype=TD)).sum().backward()
    return {k: p[k].grad.numpy() for k in KEYS}


def composite_vjp(planes: np.ndarray, d: Decisions, cam, d_out: np.ndarray) -> np.ndarray:
    """Gradient w.r.t. the planes of <d_out, composite(planes)> (the composite's VJP)."""
    pt = torch.tensor(np.asarray(planes, np.float64), dtype=TD, requires_grad=True)
    (composite_of(pt, d, cam) * torch.as_tensor(d_out, dtype=TD)).sum().backward()
    return pt.grad.numpy()


def texel_vjp_local(scene: dict, cam, part: partition.Partition, texels: np.ndarray, cot: np.ndarray,
                    ambiguous: np.ndarray | None = None) -> dict:
    """Gradient w.r.t. every Gaussian parameter of sum_j <cot_j, plane texel j> for a few plane
    texels ``texels`` [m, 3] = (k, y, x) with cotangents ``cot`` [m, 4] (dense arrays, zero for
    Gaussians that touch none of them).  Each texel is blended from all Gaussians of its chunk
    in (key, index) order with the frozen inclusion and clamp decisions taken at these
    parameters, so the cost is local: it serves full-size checks.  If ``ambiguous`` (bool [N])
    is given, Gaussians whose inclusion (o G vs 1/255) or clamp (o G vs 0.99) decision at one
    of these texels lies within float32 rounding of the threshold are flagged in it."""
    g = geometry.derive(cam)
    out = {k: np.zeros(np.asarray(scene[k]).shape) for k in KEYS}
    texels = np.asarray(texels, dtype=np.int64).reshape(-1, 3)
    cot = np.asarray(cot, dtype=np.float64).reshape(-1, 4)
    for k in np.unique(texels[:, 0]):
        idx = part.order[part.chunk_start[k]:part.chunk_start[k + 1]]
        if idx.size == 0:
            continue
        sel = texels[:, 0] == k
        ty, tx = texels[sel, 1].astype(np.float64), texels[sel, 2].astype(np.float64)
        sub = {key: np.asarray(scene[key])[idx] for key in KEYS}
        p = params_of(sub)
        mean2d, conic = project_reference(p, cam, g)
        dx = torch.from_numpy(tx)[:, None] - mean2d[None, :, 0]
        dy = torch.from_numpy(ty)[:, None] - mean2d[None, :, 1]
        quad = conic[None, :, 0, 0] * dx * dx + (conic[None, :, 0, 1] + conic[None, :, 1, 0]) * dx * dy + \
            conic[None, :, 1, 1] * dy * dy
        ln_a = torch.log(p["opacity"])[None, :] - 0.5 * quad
        with torch.no_grad():
            inc = ln_a >= splat.LN_ALPHA_MIN
            clamped = torch.exp(ln_a) >= project.ALPHA_MAX
            if ambiguous is not None:
                eps = torch.from_numpy(splat.ambiguity_eps(np.linalg.inv(conic.detach().numpy())))[None, :]
                near = ((ln_a - splat.LN_ALPHA_MIN).abs() <= eps) | ((ln_a - math.log(project.ALPHA_MAX)).abs() <= eps)
                ambiguous[idx[near.any(0).numpy()]] = True
        a = torch.exp(torch.clamp(ln_a, max=0.0))
        alpha = torch.where(inc, torch.where(clamped, torch.full_like(a, project.ALPHA_MAX), a), torch.zeros_like(a))
        Tin = torch.cumprod(torch.cat([torch.ones_like(alpha[:, :1]), 1.0 - alpha[:, :-1]], 1), 1)
        C = (Tin * alpha) @ p["rgb"]
        A = 1.0 - Tin[:, -1] * (1.0 - alpha[:, -1])
        val = (torch.cat([C, A[:, None]], 1) * torch.from_numpy(cot[sel])).sum()
        val.backward()
        for key in KEYS:
            out[key][idx] += p[key].grad.numpy()
    return out


def pixel_vjp_sparse(texel_fn, depth32, cam, dx32, dy32, interp: str, pix: np.ndarray, cot: np.ndarray):
    """The composite's VJP for a few view pixels ``pix`` [n, 3] = (v, y, x) with cotangents
    ``cot`` [n, 4] on (Q_rgb, T): returns {(k, y, x): dL/d(C, A)} over the touched texels.
    ``texel_fn(k, iy, ix)`` gives plane texels [m, 4] at in-range indices.  Back to front with
    R_k = c_k + (1 - a_k) R_{k+1}, S_k = (1 - a_k) S_{k+1}, float64."""
    g = geometry.derive(cam)
    c = decisions.constants(g, cam)
    K = len(depth32)
    pc = decisions.plane_coeffs32(c, np.asarray(depth32, np.float32), np.asarray(dx32, np.float32),
                                  np.asarray(dy32, np.float32))
    pix = np.asarray(pix, dtype=np.int64).reshape(-1, 3)
    cot = np.asarray(cot, dtype=np.float64).reshape(-1, 4)
    n = pix.shape[0]
    nearest = interp == "nearest"
    taps_all, vals = [], []
    for k in range(K):
        X = np.empty(n, dtype=np.float32)
        Y = np.empty(n, dtype=np.float32)
        for v in np.unique(pix[:, 0]):
            s = pix[:, 0] == v
            X[s], Y[s] = decisions.texel_coords32(pc, c, k, int(v), pix[s, 2], pix[s, 1], nearest)
        if nearest:
            taps = [(np.floor(Y).astype(np.int64), np.floor(X).astype(np.int64), np.ones(n))]
        else:
            x0, y0 = np.floor(X), np.floor(Y)
            wx, wy = X.astype(np.float64) - x0, Y.astype(np.float64) - y0
            x0, y0 = x0.astype(np.int64), y0.astype(np.int64)
            taps = [(y0 + oy, x0 + ox, fy * fx) for oy, fy in ((0, 1 - wy), (1, wy)) for ox, fx in ((0, 1 - wx), (1, wx))]
        s = np.zeros((n, 4))
        for iy, ix, w in taps:
            ok = (iy >= 0) & (iy < g.hp) & (ix >= 0) & (ix < g.wp)
            if np.any(ok):
                s[ok] += w[ok, None] * texel_fn(k, iy[ok], ix[ok])
        taps_all.append(taps)
        vals.append(s)
    T = np.ones(n)
    Ts = []
    for k in range(K):
        Ts.append(T.copy())
        T = T * (1.0 - vals[k][:, 3])
    R = np.zeros((n, 3))
    S = np.ones(n)
    out = {}
    for k in range(K - 1, -1, -1):
        s = vals[k]
        gc = Ts[k][:, None] * cot[:, :3]
        ga = -Ts[k] * ((cot[:, :3] * R).sum(1) + cot[:, 3] * S)
        for iy, ix, w in taps_all[k]:
            ok = (iy >= 0) & (iy < g.hp) & (ix >= 0) & (ix < g.wp) & (w != 0.0)
            for j in np.nonzero(ok)[0]:
                key = (k, int(iy[j]), int(ix[j]))
                gv = np.concatenate([w[j] * gc[j], [w[j] * ga[j]]])
                out[key] = out.get(key, 0.0) + gv
        R = s[:, :3] + (1.0 - s[:, 3])[:, None] * R
        S = (1.0 - s[:, 3]) * S
    return out


def footprint_fd(scene: dict, cam, part: partition.Partition, planes: np.ndarray, dx32, dy32, target: np.ndarray,
                 i: int, key: str, j, h: float, interp: str = "nearest"):
    """Central difference (L(theta + h e) - L(theta - h e)) / 2h of the frozen-decision loss
    L = sum (Q - Q*)^2 (views, pixels, RGB) for parameter ``key``[i, j] (j None for opacity),
    evaluated only where it can change: Gaussian i's frozen support in its plane k (the texels
    where o G >= 1/255 at theta) and the view pixels whose samples reach those texels.  Every
    other texel comes from ``planes`` [K,H,W,4] (the oracle's planes at theta), so a
    full-size workload costs a footprint, not a frame.  Within the footprint the chunk's
    Gaussians blend front to back with their inclusion and 0.99-clamp decisions frozen at
    theta, as ``frozen_loss`` does.  Returns (fd, ambiguous): ambiguous is True when some
    Gaussian's inclusion or clamp decision at a footprint texel lies within float32
    rounding of its threshold (a float32 forward may then take the other piece).  Returns
    (fd, ambiguous, support): support is False, and fd 0, when Gaussian i is culled or
    includes no texel (o G < 1/255 everywhere)."""
    g = geometry.derive(cam)
    k = int(part.chunk_of[i])
    if k < 0:
        return 0.0, False, False
    idx = part.order[part.chunk_start[k]:part.chunk_start[k + 1]]
    pr = project.project_reference(scene, np.array([i]), cam, g)
    hx, hy, ok = splat.support_halfwidth(pr, np.zeros(1))
    if not ok[0]:
        return 0.0, False, False
    mx, my = pr.mean2d[0]
    x0, x1 = max(0, math.ceil(mx - hx[0])), min(g.wp - 1, math.floor(mx + hx[0]))
    y0, y1 = max(0, math.ceil(my - hy[0])), min(g.hp - 1, math.floor(my + hy[0]))
    if x0 > x1 or y0 > y1:
        return 0.0, False, False
    yy, xx = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
    ty, tx = yy.reshape(-1), xx.reshape(-1)
    # the chunk's Gaussians whose support box meets the footprint box (the others add
    # nothing there), in (key, index) order
    pa = project.project_reference(scene, idx, cam, g)
    ax, ay, aok = splat.support_halfwidth(pa, np.zeros(idx.size))
    near = aok & (pa.mean2d[:, 0] + ax >= x0) & (pa.mean2d[:, 0] - ax <= x1) & \
        (pa.mean2d[:, 1] + ay >= y0) & (pa.mean2d[:, 1] - ay <= y1)
    sub_idx = idx[near]
    pos = int(np.nonzero(sub_idx == i)[0][0])
    sub = {kk: np.asarray(scene[kk], np.float64)[sub_idx] for kk in KEYS}

    def ln_alpha(p):
        mean2d, conic = project_reference(p, cam, g)
        ddx = torch.from_numpy(tx.astype(np.float64))[:, None] - mean2d[None, :, 0]
        ddy = torch.from_numpy(ty.astype(np.float64))[:, None] - mean2d[None, :, 1]
        quad = conic[None, :, 0, 0] * ddx * ddx + (conic[None, :, 0, 1] + conic[None, :, 1, 0]) * ddx * ddy + \
            conic[None, :, 1, 1] * ddy * ddy
        return torch.log(p["opacity"])[None, :] - 0.5 * quad, conic

    with torch.no_grad():
        p0 = params_of(sub, requires_grad=False)
        ln0, conic0 = ln_alpha(p0)
        inc = ln0 >= splat.LN_ALPHA_MIN
        clamped = ln0 >= math.log(project.ALPHA_MAX)
        eps = torch.from_numpy(splat.ambiguity_eps(np.linalg.inv(conic0.numpy())))[None, :]
        amb = bool((((ln0 - splat.LN_ALPHA_MIN).abs() <= eps) |
                    ((ln0 - math.log(project.ALPHA_MAX)).abs() <= eps)).any())
        foot = inc[:, pos].numpy()                       # the frozen support of Gaussian i
        if not foot.any():
            return 0.0, amb, False

        def texels(sign):
            p = params_of(sub, requires_grad=False)
            if j is None:
                p[key][pos] += sign * h
            else:
                p[key][pos, j] += sign * h
            ln, _ = ln_alpha(p)
            a = torch.exp(torch.clamp(ln, max=0.0))
            alpha = torch.where(inc, torch.where(clamped, torch.full_like(a, project.ALPHA_MAX), a), torch.zeros_like(a))
            Tin = torch.cumprod(torch.cat([torch.ones_like(alpha[:, :1]), 1.0 - alpha[:, :-1]], 1), 1)
            C = (Tin * alpha) @ p["rgb"]
            A = 1.0 - Tin[:, -1] * (1.0 - alpha[:, -1])
            return torch.cat([C, A[:, None]], 1).numpy()

        vals = {s: texels(s) for s in (1, -1)}
    ty, tx = ty[foot], tx[foot]
    # the view pixels whose taps reach the footprint: X depends on x only and Y on y only
    c = decisions.constants(g, cam)
    depth32 = np.asarray(part.depth, np.float32)
    dx32, dy32 = np.asarray(dx32, np.float32), np.asarray(dy32, np.float32)
    pc = decisions.plane_coeffs32(c, depth32, dx32, dy32)
    nearest = interp == "nearest"
    fx0, fx1, fy0, fy1 = tx.min(), tx.max(), ty.min(), ty.max()
    xs_all, ys_all = np.arange(cam.nx), np.arange(cam.ny)
    pix = []
    for v in range(len(dx32)):
        X, _ = decisions.texel_coords32(pc, c, k, v, xs_all, np.zeros(cam.nx, np.int64), nearest)
        _, Y = decisions.texel_coords32(pc, c, k, v, np.zeros(cam.ny, np.int64), ys_all, nearest)
        ix, iy = np.floor(X).astype(np.int64), np.floor(Y).astype(np.int64)
        reach = 0 if nearest else 1                      # bilinear also reads the next texel
        xs = xs_all[(ix + reach >= fx0) & (ix <= fx1)]
        ys = ys_all[(iy + reach >= fy0) & (iy <= fy1)]
        if xs.size and ys.size:
            gy, gx = np.meshgrid(ys, xs, indexing="ij")
            pix.append(np.stack([np.full(gx.size, v), gy.reshape(-1), gx.reshape(-1)], 1))
    if not pix:
        return 0.0, amb, True
    pix = np.concatenate(pix)
    tgt = np.asarray(target, np.float64)[pix[:, 0], pix[:, 1], pix[:, 2], :3]

    def loss(sign):
        plane_k = np.array(planes[k], np.float64)
        plane_k[ty, tx] = vals[sign][foot]
        no = np.zeros(0, bool)

        def texel_fn(kk, iy, ix):
            src = plane_k if kk == k else planes[kk]
            return np.asarray(src[iy, ix], np.float64), np.zeros(iy.shape, bool) if iy.size else no

        Q, _ = composite.composite_at(texel_fn, depth32, cam, g, dx32, dy32, interp, pix)
        return float(((Q[:, :3] - tgt) ** 2).sum())

    return (loss(1) - loss(-1)) / (2.0 * h), amb, True
