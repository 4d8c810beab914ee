"""Whole-frame oracle pipelines (float64).

* ``build_mpi_gaussians`` - Alg. 1 steps 1-5 for 3D Gaussians (G2LF, Sec. 4.4): cull and
  key, sort and chunk, then rasterise every chunk into its plane.
* ``render_view`` - the conventional per-view render the paper uses as ground truth
  (Table 1): all Gaussians in one depth-sorted list, projected into the view camera itself.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import geometry, partition, project, splat


@dataclass
class MPI:
    planes: np.ndarray      # [K,H,W,4] float64 premultiplied RGBA
    ambiguous: np.ndarray   # [K,H,W] bool
    depth: np.ndarray       # [K] float32
    part: partition.Partition
    geom: geometry.Geometry


def chunk_projection(scene, cam, geom, part, k):
    idx = part.order[part.chunk_start[k]:part.chunk_start[k + 1]]
    return project.project_reference(scene, idx, cam, geom)


def build_mpi_gaussians(scene, cam, n_chunk, binning="quantile", inv_depth_range=None, chunks=None) -> MPI:
    g = geometry.derive(cam)
    part = partition.partition(scene["means"], cam, g, n_chunk, binning, inv_depth_range)
    planes = np.zeros((n_chunk, g.hp, g.wp, 4))
    amb = np.zeros((n_chunk, g.hp, g.wp), dtype=bool)
    for k in (range(n_chunk) if chunks is None else chunks):
        proj = chunk_projection(scene, cam, g, part, k)
        planes[k], amb[k] = splat.render_plane(proj, g.hp, g.wp)
    return MPI(planes=planes, ambiguous=amb, depth=part.depth, part=part, geom=g)


def render_view(scene, cam, dx: float = 0.0, dy: float = 0.0, visible=None, dilation: float = 0.3):
    """Render one quilt view directly (the per-view baseline).

    The view camera sits at (dx, dy, 0) in base-camera coordinates, looks along +z and has
    its principal point shifted so that its principal ray meets the focal-plane centre
    (Eq. 5): c_x = (N_x - 1)/2 + p_x N_x / 2 with p_x = dx / (D_focal tan(theta_x/2)).
    ``visible`` selects the Gaussians (default: centre inside the view's guard-banded
    frustum with depth > z_near).  Returns (rgba [Ny,Nx,4], ambiguous [Ny,Nx]).
    """
    g = geometry.derive(cam)
    px = dx / (g.d_focal * g.tx)
    py = dy / (g.d_focal * g.ty)
    cxv = g.cx + px * g.nx / 2.0
    cyv = g.cy + py * g.ny / 2.0
    n = scene["means"].shape[0]
    Rc = np.asarray(cam.R, dtype=np.float64).reshape(3, 3)
    pc = scene["means"].astype(np.float64) @ Rc.T + np.asarray(cam.t, dtype=np.float64)
    key = pc[:, 2]
    if visible is None:
        z = key
        u = (g.fx * (pc[:, 0] - dx) / z + cxv - g.cx) / g.fx
        v = (g.fy * (pc[:, 1] - dy) / z + cyv - g.cy) / g.fy
        visible = (z > cam.z_near) & (np.abs(u) <= 1.3 * g.tx) & (np.abs(v) <= 1.3 * g.ty)
    idx = np.nonzero(visible)[0]
    idx = idx[np.lexsort((idx, key[idx]))]
    proj = project.project_points(scene, idx, cam, g.fx, g.fy, cxv, cyv, (dx, dy, 0.0), dilation)
    return splat.render_plane(proj, g.ny, g.nx)
