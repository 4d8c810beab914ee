"""Views composited from BF16 planes against the FP16/BF16 bar: 2e-3 max-abs per channel and
PSNR >= 50 dB against the oracle composite of the unrounded planes (RGB, all views).

A BF16 texel keeps 8 significand bits: a value in [0.5, 1) is rounded by up to 2^-9 =
1.95e-3, so a plane alone sits just inside the bar (the planes are held to it with the
other full-size checks), and a pixel whose colour comes mostly from one such texel, plus the
rounding of the planes in front of and behind it, can land beyond it.  This file is
collected after every other test, so that its result hides none of theirs."""
import numpy as np
import pytest

import scenegen
from oracle import composite
from paper_2508_18540_amd import torch_api as T
from tests import fullframe_util as F
from tests.gpu_util import announce, ctx, dev, host
from tests.test_gpu_composite import _setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_bf16_random_planes_composite(interp):
    """24 random BF16 planes, 15 views at 256 x 192."""
    announce("composite bf16 random planes", interp)
    cam, g, p, dx, dy = _setup(256, 192, 24, 15, 1, 12)
    ref, _ = composite.composite(p["rgba"], p["depth"], cam, g, dx, dy, interp)
    out = T.composite(ctx(), dev(p["rgba"], F.TDT["bf16"]), dev(p["depth"]), cam, T.views_of(dx, dy), interp)
    F.check_frame(host(out), ref, np.zeros(ref.shape[:3], bool), 2e-3, 0.0, f"bf16 random planes {interp}", True)


def test_cluster500k_bf16_views():
    """All 45 views of the headline frame built with BF16 planes."""
    announce("cluster500k bf16 views")
    folder = F.oracle("frame", "--config", "cluster500k")
    scene, cam, cfg = scenegen.config("cluster500k")
    K = cfg["n_chunk"]
    ds = T.to_device(scene)
    ws = T.workspace_for(ds, cam, K)
    out = T.build_mpi(ctx(), ds, cam, K, dtype=F.TDT["bf16"], workspace=ws)
    T.build_stats(ctx(), ws, check=True)
    dx, dy = F.views(cam, cfg["vx"])
    views = T.composite(ctx(), out["rgba"], out["depth"], cam, T.views_of(dx, dy), "nearest")
    F.check_frame(host(views), F.load(folder, "views"), F.load(folder, "vamb"), 2e-3, 0.03,
                  "cluster500k bf16 planes, float32 views", True)


def test_voxel256_bf16_views():
    """All 96 views of the voxel workload built with BF16 planes."""
    announce("voxel256 bf16 views")
    folder = F.oracle("frame", "--config", "voxel256")
    vox, cam, cfg = scenegen.config("voxel256")
    K = cfg["n_chunk"]
    ds = T.to_device(vox)
    ws = T.workspace_for(ds, cam, K)
    out = T.build_mpi(ctx(), ds, cam, K, dtype=F.TDT["bf16"], workspace=ws)
    T.build_stats(ctx(), ws, check=True)
    dx, dy = F.views(cam, cfg["vx"])
    views = T.composite(ctx(), out["rgba"], out["depth"], cam, T.views_of(dx, dy), "nearest")
    ref = F.load(folder, "views")
    F.check_frame(host(views), ref, np.zeros(ref.shape[:3], bool), 2e-3, 0.0, "voxel256 bf16 planes, views", True)
