"""The pooled whole-frame oracle runner returns exactly what the single-process oracle
computes (it only spreads planes and views over worker processes)."""
import os
import subprocess
import sys

import numpy as np

import scenegen
from oracle import composite, geometry, pool, render, voxels

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pool_frame_equals_serial_oracle():
    scene, cam, cfg = scenegen.config("uniform10k")
    dx, dy, _, _ = geometry.quilt_views(cam, 5, 1)
    dx, dy = dx.astype(np.float32), dy.astype(np.float32)
    res, t = pool.frame(scene, cam, 16, "gaussians", "inv_depth", (2.0, 6.0), dx, dy, "bilinear", processes=3)
    mpi = render.build_mpi_gaussians(scene, cam, 16, "inv_depth", (2.0, 6.0))
    assert np.array_equal(res["planes"], mpi.planes) and np.array_equal(res["amb"], mpi.ambiguous)
    assert np.array_equal(res["chunk_of"], mpi.part.chunk_of)
    ref, amb = composite.composite(mpi.planes, mpi.depth, cam, mpi.geom, dx, dy, "bilinear", mpi.ambiguous)
    assert np.array_equal(res["views"], ref) and np.array_equal(res["vamb"], amb)
    assert t["processes"] == 3


def test_pool_voxel_planes_equal_serial_oracle():
    vox = scenegen.voxel_scene(res=16, n_occupied=300, seed=5)
    cam = scenegen.camera(48, 40, 50.0, 4.0, 0.5)
    res, _ = pool.frame(vox, cam, 4, "voxels", processes=2)
    mpi = voxels.build_mpi_voxels(vox, cam, 4)
    assert np.array_equal(res["planes"], mpi.planes) and not res["amb"].any()


def test_pool_program_writes_frame(tmp_path):
    r = subprocess.run([sys.executable, "-m", "oracle.pool", "frame", "--config", "uniform10k", "--out", str(tmp_path),
                        "--processes", "2"], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    views = np.load(tmp_path / "views.npy")
    assert views.shape == (9, 128, 128, 4) and np.all((views[..., 3] >= 0) & (views[..., 3] <= 1))
