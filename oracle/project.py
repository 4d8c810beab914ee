"""EWA projection of 3D Gaussians into the reference camera, float64 (Sec. 4.4).

The reference camera sits at (0, 0, D_forward) in base-camera coordinates with the
base camera's orientation and the field of view theta' of Eq. 2; its image is the
W_p x H_p plane grid.  A Gaussian with mean m, log-scales l and rotation quaternion
q (w, x, y, z; normalised here) has world covariance Sigma = R(q) diag(e^{2l}) R(q)^T.
With p = R_cam m + t_cam and z = p_z - D_forward the projected mean and covariance are

    mu' = (f'_x p_x / z + c'_x,  f'_y p_y / z + c'_y)
    Sigma' = J W Sigma W^T J^T + f' I,   J = [[f'_x/z, 0, -f'_x p_x/z^2], [0, f'_y/z, -f'_y p_y/z^2]]

with W = R_cam and f' the adaptive dilation of Eq. 8.  A texel at p contributes
alpha = min(0.99, o G(p)), G(p) = exp(-1/2 (p - mu')^T Sigma'^-1 (p - mu')), and only
where o G(p) >= 1/255 (the inclusion rule of the 3DGS rasteriser the method extends).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [N,3,3] of quaternions (w, x, y, z), normalised first."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


@dataclass
class Projected:
    mean2d: np.ndarray    # [n,2] texel coordinates
    cov2d: np.ndarray     # [n,2,2] Sigma' including the dilation
    conic: np.ndarray     # [n,2,2] inverse of cov2d
    depth: np.ndarray     # [n] z relative to the projecting camera
    opacity: np.ndarray   # [n]
    rgb: np.ndarray       # [n,3]


def world_covariance(log_scales, quats) -> np.ndarray:
    R = quat_to_rot(quats)
    s2 = np.exp(2.0 * np.asarray(log_scales, dtype=np.float64))
    return np.einsum("nij,nj,nkj->nik", R, s2, R)


def project_points(scene: dict, idx, cam, fx, fy, cx, cy, cam_pos, dilation) -> Projected:
    """Project Gaussians ``idx`` into a pinhole camera at ``cam_pos`` (base-camera coordinates)
    with the base camera's orientation, focal lengths fx, fy and principal point cx, cy."""
    idx = np.asarray(idx, dtype=np.int64)
    Rc = np.asarray(cam.R, dtype=np.float64).reshape(3, 3)
    tc = np.asarray(cam.t, dtype=np.float64)
    m = scene["means"][idx].astype(np.float64)
    p = m @ Rc.T + tc - np.asarray(cam_pos, dtype=np.float64)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    mean2d = np.stack([fx * x / z + cx, fy * y / z + cy], axis=1)
    sig = world_covariance(scene["log_scales"][idx], scene["quats"][idx])
    sig_c = np.einsum("ij,njk,lk->nil", Rc, sig, Rc)
    J = np.zeros((idx.size, 2, 3))
    J[:, 0, 0] = fx / z
    J[:, 0, 2] = -fx * x / (z * z)
    J[:, 1, 1] = fy / z
    J[:, 1, 2] = -fy * y / (z * z)
    cov = np.einsum("nij,njk,nlk->nil", J, sig_c, J) + dilation * np.eye(2)[None]
    conic = np.linalg.inv(cov)
    return Projected(mean2d=mean2d, cov2d=cov, conic=conic, depth=z,
                     opacity=scene["opacity"][idx].astype(np.float64),
                     rgb=scene["rgb"][idx].astype(np.float64))


def project_reference(scene: dict, idx, cam, g) -> Projected:
    """Projection into the reference camera (Eqs. 1-2, 8)."""
    return project_points(scene, idx, cam, g.fpx, g.fpy, g.cpx, g.cpy, (0.0, 0.0, g.d_forward),
                          g.f_dilation)
