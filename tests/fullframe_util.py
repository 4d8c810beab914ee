"""Shared helpers of the whole-workload GPU tests: the pooled oracle program run once per
argument list in this process, and the frame comparisons against the bars."""
import os
import subprocess
import sys
import tempfile

import numpy as np
import torch

from oracle import geometry
from tests.gpu_util import psnr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TDT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
_FRAMES = {}


def oracle(*args, key=None):
    """Runs the pooled oracle program once per argument list; returns its output folder."""
    key = key or args
    if key in _FRAMES:
        return _FRAMES[key]
    out = tempfile.mkdtemp(prefix="lf_oracle_")
    print("[oracle]", *args, flush=True)
    r = subprocess.run([sys.executable, "-m", "oracle.pool", *args, "--out", out], cwd=ROOT, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    print(r.stdout.strip(), flush=True)
    _FRAMES[key] = out
    return out


def load(folder, name):
    return np.load(os.path.join(folder, name + ".npy"), mmap_mode="r")


def masked_stats(got, ref, amb):
    """Per-texel max channel error split by the ambiguity mask."""
    err = np.abs(got - ref).max(axis=-1)
    return err, float(err[~amb].max(initial=0.0)), float(err[amb].max(initial=0.0)), float(amb.mean())


def check_frame(got, ref, amb, tol, jump, what, low_precision):
    """got/ref [..., 4]; every unmasked element within tol, masked ones within jump, and for
    low-precision planes PSNR >= 50 dB over the RGB of every element."""
    err, e_un, e_amb, frac = masked_stats(got, ref, amb)
    q = psnr(got[..., :3], ref[..., :3]) if low_precision else None
    print(f"{what}: unmasked max-abs {e_un:.3e} (bar {tol:g}), ambiguous fraction {frac:.2e} max {e_amb:.3e}"
          + (f", PSNR {q:.2f} dB" if q is not None else ""), flush=True)
    bad = (err > tol) & ~amb
    assert not bad.any(), f"{what}: {int(bad.sum())} unmasked elements above {tol}: max {e_un}"
    assert e_amb <= jump, f"{what}: ambiguous elements up to {e_amb}"
    if q is not None:
        assert q >= 50.0, f"{what}: PSNR {q}"
    return frac


def check_partition(out, folder, n):
    torch.cuda.synchronize()
    assert np.array_equal(out["chunk_of"].cpu().numpy()[:n], load(folder, "chunk_of"))
    assert np.array_equal(out["chunk_count"].cpu().numpy(), load(folder, "chunk_count"))
    assert np.array_equal(out["depth"].cpu().numpy().view(np.uint32), np.asarray(load(folder, "depth")).view(np.uint32))


def views(cam, vx, vy=1):
    dx, dy, _, _ = geometry.quilt_views(cam, vx, vy)
    return dx.astype(np.float32), dy.astype(np.float32)


