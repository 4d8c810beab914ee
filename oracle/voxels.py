"""Sparse-voxel fields rendered into sweeping planes (V2LF, Sec. 4.5; Alg. 1 with voxels).

Test infrastructure (float64).  A voxel is an axis-aligned world cube
``origin + h * ([i, i+1] x [j, j+1] x [k, k+1])`` holding eight corner densities (per world
unit; corner bit 0 = +x, bit 1 = +y, bit 2 = +z) with trilinear interpolation inside, and an
RGB colour.  Sec. 4.5 treats voxels like Gaussians: a discrete primitive set that is culled,
depth-sorted and chunked by the same rules (``partition``), then rasterised chunk by chunk
into the reference camera's planes; instead of a prefilter, a low-pass filter runs over the
finished planes in place.

Readings where the paper is silent:
* a voxel's depth key is the base-camera z of its centre; the centre is the float32 program
  ``fl(o + fl(h * fl(i + 1/2)))`` per axis, so both implementations key identical bits;
* per plane texel, the reference ray ``p(t) = (0, 0, D_forward) + t r`` with
  ``r = ((X - c'_x)/f'_x, (Y - c'_y)/f'_y, 1)`` (base-camera coordinates, t >= 0) crosses each
  voxel of the chunk over its slab interval [t0, t1]; the optical depth is
  ``tau = |r| * integral_{t0}^{t1} rho(p(t)) dt`` (exact: the trilinear density restricted to
  a line is a cubic in t), alpha = 1 - exp(-tau) with no clamp and no threshold, and the
  voxels of a chunk are blended front to back in (key, index) order, C += T alpha rgb,
  T *= 1 - alpha; the plane stores (C, 1 - T);
* the low-pass filter is the separable binomial [1, 2, 1] / 4 on every channel of the
  premultiplied planes, with zero padding outside the plane.
"""
from __future__ import annotations

import numpy as np

from . import geometry, partition
from .render import MPI

F = np.float32

# 3-point Gauss-Legendre rule on [-1, 1]: exact for polynomials of degree <= 5
_GL3_X = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_GL3_W = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def centres32(ijk: np.ndarray, origin, h: float) -> np.ndarray:
    """Voxel centres in float32: fl(o + fl(h * fl(i + 1/2))) per axis."""
    half = ijk.astype(np.float32) + F(0.5)
    return (np.asarray(origin, dtype=np.float32)[None, :] + F(h) * half).astype(np.float32)


def trilinear(dens: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Trilinear density at local coordinates u [..., 3] in [0, 1]^3 from corners dens [..., 8]."""
    out = np.zeros(u.shape[:-1])
    for c in range(8):
        w = np.ones(u.shape[:-1])
        for axis in range(3):
            w = w * (u[..., axis] if (c >> axis) & 1 else 1.0 - u[..., axis])
        out = out + dens[..., c] * w
    return out


def slab(a: np.ndarray, b: np.ndarray):
    """Parameter interval [t0, t1] (t >= 0) where a + t b lies in [0, 1]^3; a, b [..., 3]."""
    t0 = np.zeros(a.shape[:-1])
    t1 = np.full(a.shape[:-1], np.inf)
    for axis in range(3):
        ai, bi = a[..., axis], b[..., axis]
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (0.0 - ai) / bi
            tb = (1.0 - ai) / bi
        lo = np.where(bi != 0.0, np.minimum(ta, tb), np.where((ai >= 0.0) & (ai <= 1.0), -np.inf, np.inf))
        hi = np.where(bi != 0.0, np.maximum(ta, tb), np.where((ai >= 0.0) & (ai <= 1.0), np.inf, -np.inf))
        t0 = np.maximum(t0, lo)
        t1 = np.minimum(t1, hi)
    return t0, t1


def optical_depth(dens: np.ndarray, a: np.ndarray, b: np.ndarray, rnorm: np.ndarray) -> np.ndarray:
    """tau = |r| * integral of the trilinear density along a + t b over its slab interval."""
    t0, t1 = slab(a, b)
    hit = t1 > t0
    tau = np.zeros(a.shape[:-1])
    if not np.any(hit):
        return tau
    t0h, t1h = t0[hit], t1[hit]
    mid, half = 0.5 * (t0h + t1h), 0.5 * (t1h - t0h)
    acc = np.zeros(mid.shape)
    for x, w in zip(_GL3_X, _GL3_W):
        t = mid + half * x
        u = np.clip(a[hit] + t[:, None] * b[hit], 0.0, 1.0)
        acc = acc + w * trilinear(np.broadcast_to(dens, u.shape[:-1] + (8,)), u)
    tau[hit] = rnorm[hit] * half * acc
    return tau


def _camera(cam):
    R = np.asarray(cam.R, dtype=np.float64).reshape(3, 3)
    t = np.asarray(cam.t, dtype=np.float64)
    return R, t


def texel_rays(g: geometry.Geometry, xs: np.ndarray, ys: np.ndarray):
    """Reference-camera ray directions r (base-camera coordinates, r_z = 1) of texels (xs, ys)."""
    r = np.stack([(xs - g.cpx) / g.fpx, (ys - g.cpy) / g.fpy, np.ones(np.shape(xs))], axis=-1)
    return r


def support_rect(lo_world: np.ndarray, h: float, cam, g: geometry.Geometry):
    """Texel rectangle (x0, y0, x1, y1) holding every texel whose ray can meet the voxel."""
    R, t = _camera(cam)
    corners = np.array([[(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.float64)
    pc = (lo_world[None, :] + h * corners) @ R.T + t
    zr = pc[:, 2] - g.d_forward
    if np.any(zr <= 0.0):
        return 0, 0, g.wp - 1, g.hp - 1
    X = g.fpx * pc[:, 0] / zr + g.cpx
    Y = g.fpy * pc[:, 1] / zr + g.cpy
    x0, x1 = max(int(np.floor(X.min())), 0), min(int(np.ceil(X.max())), g.wp - 1)
    y0, y1 = max(int(np.floor(Y.min())), 0), min(int(np.ceil(Y.max())), g.hp - 1)
    return x0, y0, x1, y1


def render_plane(vox: dict, idx: np.ndarray, cam, g: geometry.Geometry) -> np.ndarray:
    """One plane: the voxels ``idx`` (in blending order) rasterised front to back -> [H,W,4]."""
    R, t = _camera(cam)
    origin = np.asarray(vox["origin"], dtype=np.float64)
    h = float(vox["voxel_size"])
    ray_origin_world = R.T @ (np.array([0.0, 0.0, g.d_forward]) - t)
    C = np.zeros((g.hp, g.wp, 3))
    T = np.ones((g.hp, g.wp))
    for i in idx:
        lo = origin + h * vox["ijk"][i].astype(np.float64)
        x0, y0, x1, y1 = support_rect(lo, h, cam, g)
        if x0 > x1 or y0 > y1:
            continue
        ys, xs = np.meshgrid(np.arange(y0, y1 + 1, dtype=np.float64), np.arange(x0, x1 + 1, dtype=np.float64),
                             indexing="ij")
        r = texel_rays(g, xs, ys)
        a = np.broadcast_to((ray_origin_world - lo) / h, r.shape)
        b = (r @ R) / h                                    # R^T r per texel, in voxel units
        tau = optical_depth(vox["density"][i].astype(np.float64), a, b, np.linalg.norm(r, axis=-1))
        alpha = 1.0 - np.exp(-tau)
        Tw = T[y0:y1 + 1, x0:x1 + 1]
        C[y0:y1 + 1, x0:x1 + 1] += (alpha * Tw)[..., None] * vox["rgb"][i].astype(np.float64)[None, None, :]
        T[y0:y1 + 1, x0:x1 + 1] = Tw * (1.0 - alpha)
    return np.concatenate([C, (1.0 - T)[..., None]], axis=-1)


def lowpass(plane: np.ndarray) -> np.ndarray:
    """Separable [1, 2, 1] / 4 filter of a [H, W, C] plane, zero outside the plane."""
    p = np.pad(plane, ((1, 1), (1, 1), (0, 0)))
    rows = 0.25 * p[:-2] + 0.5 * p[1:-1] + 0.25 * p[2:]
    return 0.25 * rows[:, :-2] + 0.5 * rows[:, 1:-1] + 0.25 * rows[:, 2:]


def partition_voxels(vox: dict, cam, g, n_chunk: int, binning="quantile", inv_depth_range=None):
    return partition.partition(centres32(vox["ijk"], vox["origin"], vox["voxel_size"]), cam, g, n_chunk, binning,
                               inv_depth_range)


def build_mpi_voxels(vox: dict, cam, n_chunk: int, binning="quantile", inv_depth_range=None, chunks=None,
                     filtered: bool = True) -> MPI:
    """Alg. 1 steps 1-5 for sparse voxels: cull and key the centres, sort and chunk,
    rasterise every chunk, then low-pass every plane."""
    g = geometry.derive(cam)
    part = partition_voxels(vox, cam, g, n_chunk, binning, inv_depth_range)
    planes = np.zeros((n_chunk, g.hp, g.wp, 4))
    for k in (range(n_chunk) if chunks is None else chunks):
        idx = part.order[part.chunk_start[k]:part.chunk_start[k + 1]]
        planes[k] = render_plane(vox, idx, cam, g)
        if filtered:
            planes[k] = lowpass(planes[k])
    return MPI(planes=planes, ambiguous=np.zeros((n_chunk, g.hp, g.wp), dtype=bool), depth=part.depth, part=part,
               geom=g)


__all__ = ["centres32", "trilinear", "slab", "optical_depth", "texel_rays", "support_rect", "render_plane",
           "lowpass", "partition_voxels", "build_mpi_voxels"]
