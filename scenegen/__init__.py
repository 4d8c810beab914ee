"""Seeded synthetic inputs: radiance fields, display/camera settings and plane stacks.

This module is the only code shared by the FP64 oracle (``oracle/``) and the
GPU path (``paper_2508_18540_amd``).  It holds none of the method's
arithmetic: it draws random numbers and states the workload parameters
(resolution, plane count, view count, display angles).  Everything derived
from them (reference camera, view offsets, plane depths, footprints) is
computed separately by each side.

All random draws use ``numpy.random.Generator(PCG64(seed))``.  Arrays are
returned as C-contiguous float32 (int32 for voxel indices), the precision in
which both sides receive them.

Workloads (the paper evaluates on trained MipNeRF-360 models, which are not
available; these seeded scenes stand in for them with the shapes, sizes and
depth structure of its experiments):

* ``uniform_scene``   10,000 Gaussians, means uniform in [-1,1]^2 x [2,6].
* ``cluster_scene``   Gaussians from a 64-cluster mixture over depth 1..20.
* ``voxel_scene``     256^3 grid, 2 % occupancy from thresholded value noise.
* ``random_planes``   premultiplied RGBA plane stacks for compositing tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

__all__ = [
    "Camera", "camera", "uniform_scene", "cluster_scene", "voxel_scene",
    "random_planes", "perturbed_target", "small_scene", "CONFIGS", "config", "config_camera",
    "BATCH_SCENES", "batch_scene",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


@dataclass(frozen=True)
class Camera:
    """Base camera plus display settings, every field already rounded to float32.

    ``R``/``t`` map world points to base-camera coordinates (x right, y down,
    looking along +z).  Angles are full angles in radians.
    """
    R: tuple
    t: tuple
    nx: int
    ny: int
    fov_x: float
    fov_y: float
    d_focal: float
    phi_x: float
    phi_y: float
    d_shift: float = 0.0
    plane_scale: float = 1.0
    z_near: float = 0.2
    dilation: float = 0.0     # f' in reference texels^2; 0 = the adaptive value of Eq. 8

    def with_(self, **kw) -> "Camera":
        kw = {k: (float(np.float32(v)) if isinstance(v, float) else v) for k, v in kw.items()}
        return replace(self, **kw)


def camera(nx: int, ny: int, fov_deg: float, d_focal: float, phi_x: float, phi_y: float = 0.0,
           plane_scale: float = 1.0, d_shift: float = 0.0, z_near: float = 0.2,
           R=None, t=None, fov_y_deg: float | None = None, dilation: float = 0.0) -> Camera:
    """Build a :class:`Camera`; ``phi_*`` are display viewing angles in radians."""
    R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64).reshape(3, 3)
    t = np.zeros(3) if t is None else np.asarray(t, dtype=np.float64).reshape(3)
    f = lambda v: float(np.float32(v))
    fy = fov_deg if fov_y_deg is None else fov_y_deg
    return Camera(R=tuple(f(v) for v in R.reshape(-1)), t=tuple(f(v) for v in t),
                  nx=int(nx), ny=int(ny), fov_x=f(math.radians(fov_deg)), fov_y=f(math.radians(fy)),
                  d_focal=f(d_focal), phi_x=f(phi_x), phi_y=f(phi_y), d_shift=f(d_shift),
                  plane_scale=f(plane_scale), z_near=f(z_near), dilation=f(dilation))


def _gaussian_attributes(rng: np.random.Generator, n: int, means: np.ndarray) -> dict:
    """Draw log-scales, quaternions, opacities and colours after the means."""
    log_scales = rng.normal(-3.0, 0.5, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))           # (w, x, y, z), not normalised
    logits = rng.normal(0.0, 1.0, size=n)
    rgb = rng.random(size=(n, 3))
    opacity = 1.0 / (1.0 + np.exp(-logits))
    return dict(means=_f32(means), log_scales=_f32(log_scales), quats=_f32(quats),
                opacity=_f32(opacity), rgb=_f32(rgb))


def uniform_scene(n: int = 10_000, seed: int = 0) -> dict:
    """Means uniform in [-1,1] x [-1,1] x [2,6] (depth in front of the base camera)."""
    rng = _rng(seed)
    u = rng.random(size=(n, 3))
    means = np.empty_like(u)
    means[:, 0] = -1.0 + 2.0 * u[:, 0]
    means[:, 1] = -1.0 + 2.0 * u[:, 1]
    means[:, 2] = 2.0 + 4.0 * u[:, 2]
    return _gaussian_attributes(rng, n, means)


def cluster_scene(n: int = 500_000, seed: int = 1, n_clusters: int = 64,
                  z_range=(1.0, 20.0)) -> dict:
    """Equal-weight mixture of isotropic clusters spread over depth ``z_range``.

    Cluster centre depth ~ U[1.5, 19.5], lateral centre ~ U(-0.8, 0.8) * z * tan 25deg,
    points = centre + N(0, (0.1 z_c)^2 I), depth clipped to ``z_range``.
    """
    rng = _rng(seed)
    zc = rng.uniform(1.5, 19.5, size=n_clusters)
    lat = rng.uniform(-0.8, 0.8, size=(n_clusters, 2)) * (zc * math.tan(math.radians(25.0)))[:, None]
    centres = np.stack([lat[:, 0], lat[:, 1], zc], axis=1)
    cid = rng.integers(0, n_clusters, size=n)
    offs = rng.normal(0.0, 1.0, size=(n, 3)) * (0.1 * zc[cid])[:, None]
    means = centres[cid] + offs
    means[:, 2] = np.clip(means[:, 2], z_range[0], z_range[1])
    return _gaussian_attributes(rng, n, means)


def small_scene(n: int, seed: int, xy: float = 0.6, z=(2.0, 4.0), log_scale=(-2.5, 0.4)) -> dict:
    """Tiny scenes for brute-force and edge-case tests (larger footprints)."""
    rng = _rng(seed)
    u = rng.random(size=(n, 3))
    means = np.empty_like(u)
    means[:, 0] = -xy + 2 * xy * u[:, 0]
    means[:, 1] = -xy + 2 * xy * u[:, 1]
    means[:, 2] = z[0] + (z[1] - z[0]) * u[:, 2]
    log_scales = rng.normal(log_scale[0], log_scale[1], size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    logits = rng.normal(0.5, 1.0, size=n)
    rgb = rng.random(size=(n, 3))
    opacity = 1.0 / (1.0 + np.exp(-logits))
    return dict(means=_f32(means), log_scales=_f32(log_scales), quats=_f32(quats),
                opacity=_f32(opacity), rgb=_f32(rgb))


def perturbed_target(scene: dict, seed: int) -> dict:
    """Target scene for the gradient workload: means + N(0, 0.01^2), opacity * (1 + U(-0.1, 0.1))."""
    rng = _rng(seed)
    n = scene["means"].shape[0]
    dm = rng.normal(0.0, 0.01, size=(n, 3))
    fo = 1.0 + rng.uniform(-0.1, 0.1, size=n)
    out = {k: v.copy() for k, v in scene.items()}
    out["means"] = _f32(scene["means"].astype(np.float64) + dm)
    out["opacity"] = _f32(np.clip(scene["opacity"].astype(np.float64) * fo, 1e-6, 0.9999))
    return out


def _value_noise(res: int, lattice: np.ndarray) -> np.ndarray:
    """Trilinear value noise with smoothstep weights evaluated at cell centres of a res^3 grid."""
    L = lattice.shape[0] - 1
    c = (np.arange(res, dtype=np.float64) + 0.5) / res * L
    i0 = np.minimum(np.floor(c).astype(np.int64), L - 1)
    f = c - i0
    w = f * f * (3.0 - 2.0 * f)
    out = np.empty((res, res, res), dtype=np.float64)        # [z][y][x]
    for kz in range(res):
        z0, wz = i0[kz], w[kz]
        acc = np.zeros((res, res))
        for dz, fz in ((0, 1.0 - wz), (1, wz)):
            sl = lattice[z0 + dz]                             # [y][x] lattice slice
            a = sl[i0][:, i0]
            b = sl[i0][:, i0 + 1]
            c_ = sl[i0 + 1][:, i0]
            d = sl[i0 + 1][:, i0 + 1]
            wy = w[:, None]
            wx = w[None, :]
            v = (a * (1 - wx) + b * wx) * (1 - wy) + (c_ * (1 - wx) + d * wx) * wy
            acc += fz * v
        out[kz] = acc
    return out


def voxel_scene(res: int = 256, n_occupied: int = 335_544, seed: int = 2,
                bbox=((-1.0, -1.0, 3.0), (1.0, 1.0, 5.0)), lattice_size: int = 17,
                density_median: float = 40.0, density_sigma: float = 0.5) -> dict:
    """Sparse voxels: the ``n_occupied`` cells of largest value noise (ties by linear index).

    Returns ijk [n,3] int32 (x, y, z cell indices), corner densities [n,8] (corner bit0 = +x,
    bit1 = +y, bit2 = +z, per world unit), rgb [n,3], and the grid origin / cell size.
    """
    rng = _rng(seed)
    lattice = rng.random(size=(lattice_size,) * 3)
    noise = _value_noise(res, lattice).reshape(-1)           # linear = (z*res + y)*res + x
    order = np.argsort(-noise, kind="stable")[:n_occupied]
    lin = np.sort(order)
    ix = lin % res
    iy = (lin // res) % res
    iz = lin // (res * res)
    ijk = np.stack([ix, iy, iz], axis=1).astype(np.int32)
    dens = np.exp(rng.normal(math.log(density_median), density_sigma, size=(n_occupied, 8)))
    rgb = rng.random(size=(n_occupied, 3))
    lo, hi = np.asarray(bbox[0], dtype=np.float64), np.asarray(bbox[1], dtype=np.float64)
    size = (hi - lo) / res
    assert np.allclose(size, size[0]), "voxel grid must be cubic"
    return dict(ijk=np.ascontiguousarray(ijk), density=_f32(dens), rgb=_f32(rgb),
                origin=tuple(float(np.float32(v)) for v in lo), voxel_size=float(np.float32(size[0])),
                grid_res=res)


def sh_coefficients(n: int, degree: int, seed: int, dc_range: float = 1.7, ac_scale: float = 0.4) -> np.ndarray:
    """Spherical-harmonic colour coefficients [n, (degree+1)^2, 3] float32: the DC term
    uniform in (-dc_range, dc_range), band l >= 1 normal with deviation ac_scale / l."""
    rng = _rng(seed)
    nc = (degree + 1) ** 2
    c = np.empty((n, nc, 3))
    c[:, 0] = rng.uniform(-dc_range, dc_range, size=(n, 3))
    for l in range(1, degree + 1):
        c[:, l * l:(l + 1) ** 2] = rng.normal(scale=ac_scale / l, size=(n, 2 * l + 1, 3))
    return _f32(c)


def random_planes(n_chunk: int, height: int, width: int, seed: int, depth_range=(1.5, 12.0),
                  p_empty: float = 0.3, p_opaque: float = 0.05) -> dict:
    """A premultiplied RGBA plane stack with sorted depths, for compositing tests.

    A texel is empty with probability ``p_empty``, fully opaque with ``p_opaque``,
    otherwise alpha ~ U(0,1); colour = alpha * U(0,1)^3.
    """
    rng = _rng(seed)
    u = rng.random(size=(n_chunk, height, width))
    a = rng.random(size=(n_chunk, height, width))
    a = np.where(u < p_empty, 0.0, np.where(u < p_empty + p_opaque, 1.0, a))
    c = rng.random(size=(n_chunk, height, width, 3)) * a[..., None]
    rgba = np.concatenate([c, a[..., None]], axis=-1)
    d = np.sort(rng.uniform(depth_range[0], depth_range[1], size=n_chunk))
    return dict(rgba=_f32(rgba), depth=_f32(d))


# ---------------------------------------------------------------------------------------------
# Workload table.  Each entry names a scene recipe and the display / plane settings.
# ---------------------------------------------------------------------------------------------

def _baseline_phi(baseline: float, d_focal: float) -> float:
    # A total lateral camera span of `baseline` at the focal distance spans this viewing angle.
    return 2.0 * math.atan(0.5 * baseline / d_focal)


CONFIGS = {
    # plain method, FP32: 10k uniform Gaussians, 128^2, 16 inverse-depth planes over [2,6], 9 views
    "uniform10k": dict(scene=("uniform", dict(n=10_000, seed=0)), res=128, n_chunk=16,
                       binning="inv_depth", inv_depth_range=(2.0, 6.0), vx=9, vy=1,
                       d_focal=3.0, phi_x=_baseline_phi(0.1, 3.0), fov_deg=50.0),
    # 500k clustered Gaussians, 512^2, 64 quantile planes, 45 views over +-20 deg
    "cluster500k": dict(scene=("cluster", dict(n=500_000, seed=1)), res=512, n_chunk=64,
                        binning="quantile", vx=45, vy=1, d_focal=2.0, phi_x=math.radians(40.0),
                        fov_deg=50.0),
    # 2D parallax: the cluster500k scene and planes seen by a 9 x 5 quilt over +-20 x +-10 deg
    "quilt2d": dict(scene=("cluster", dict(n=500_000, seed=1)), res=512, n_chunk=64,
                    binning="quantile", vx=9, vy=5, d_focal=2.0, phi_x=math.radians(40.0),
                    phi_y=math.radians(20.0), fov_deg=50.0),
    # sparse voxels, 512^2, 64 quantile planes, 96 views
    "voxel256": dict(scene=("voxel", dict(seed=2)), res=512, n_chunk=64, binning="quantile",
                     vx=96, vy=1, d_focal=4.0, phi_x=math.radians(40.0), fov_deg=50.0),
    # differentiation workload: 200k clustered Gaussians, 128 planes, 45 views
    "grad200k": dict(scene=("cluster", dict(n=200_000, seed=4)), res=512, n_chunk=128,
                     binning="quantile", vx=45, vy=1, d_focal=2.0, phi_x=math.radians(40.0),
                     fov_deg=50.0, target_seed=5),
}

# batched workload: (n_gaussians, resolution, n_chunk, n_views), seeds 30 + i
BATCH_SCENES = [
    (50_000, 256, 64, 9), (100_000, 384, 128, 16), (200_000, 512, 64, 45), (400_000, 768, 128, 24),
    (700_000, 256, 512, 100), (1_000_000, 384, 64, 48), (1_500_000, 512, 512, 96),
    (2_000_000, 768, 128, 45),
]


def batch_scene(i: int):
    """Scene i of the batched workload: (scene, camera, N_chunk, views per row); clustered
    Gaussians as cluster500k (seed 30 + i), D_focal = 2, 40 deg of horizontal parallax."""
    n, res, K, V = BATCH_SCENES[i]
    cam = camera(res, res, 50.0, 2.0, math.radians(40.0))
    return cluster_scene(n, seed=30 + i), cam, K, V


def config_camera(name: str, **override):
    """Return (camera, settings) of a named workload without drawing its scene."""
    c = dict(CONFIGS[name])
    c.update(override)
    cam = camera(c["res"], c["res"], c["fov_deg"], c["d_focal"], c["phi_x"], c.get("phi_y", 0.0),
                 plane_scale=c.get("plane_scale", 1.0))
    return cam, c


def config(name: str, **override):
    """Return (scene, camera, settings) for a named workload."""
    cam, c = config_camera(name, **override)
    kind, kw = c["scene"]
    if kind == "uniform":
        scene = uniform_scene(**kw)
    elif kind == "cluster":
        scene = cluster_scene(**kw)
    elif kind == "voxel":
        scene = voxel_scene(**kw)
    else:
        raise ValueError(kind)
    return scene, cam, c
