"""GPU parity of the hand-written backward (lf_composite_backward, lf_build_mpi_backward
and the LFRender autograd function) against the FP64 gradient oracle and against central
finite differences of the oracle's frozen-decision loss.

Gradient bar: |g - g_ref| <= 1e-3 max(|g_ref|, 1e-2 max_i |g_ref,i|) per parameter tensor."""
import math

import numpy as np
import pytest
import torch

import scenegen
from oracle import geometry, grad
from paper_2508_18540_amd import torch_api as T
from tests.gpu_util import announce, ctx, dev, host

pytestmark = pytest.mark.gpu


def _check(got: np.ndarray, ref: np.ndarray, name: str, rel=1e-3, floor=1e-2, allow=0):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), floor * np.abs(ref).max())
    bad = np.abs(got - ref) > rel * scale
    worst = float((np.abs(got - ref) / np.maximum(scale, 1e-300)).max())
    print(f"{name}: max |g| {np.abs(ref).max():.3e}, worst scaled error {worst:.2e}, violations {int(bad.sum())}")
    assert int(bad.sum()) <= allow, f"{name}: {int(bad.sum())} entries beyond the bar"


def _views(cam, n):
    dx, dy, _, _ = geometry.quilt_views(cam, n, 1)
    return dx.astype(np.float32), dy.astype(np.float32)


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
@pytest.mark.parametrize("pdt", [torch.float32, torch.float16])
def test_composite_backward_matches_oracle(interp, pdt):
    announce("composite backward", interp, pdt)
    cam = scenegen.camera(40, 36, 50.0, 3.0, math.radians(30.0))
    g = geometry.derive(cam)
    K = 7
    p = scenegen.random_planes(K, g.hp, g.wp, seed=11)
    dx, dy = _views(cam, 6)
    d = grad.composite_decisions(cam, p["depth"], dx, dy, interp)
    rng = np.random.default_rng(2)
    d_out = rng.normal(size=(len(dx), cam.ny, cam.nx, 4))
    rgba = dev(p["rgba"], pdt)
    depth = dev(p["depth"])
    got = host(T.composite_backward(ctx(), rgba, depth, cam, T.views_of(dx, dy), dev(d_out, torch.float32), interp))
    planes = host(rgba)                                # the planes as the GPU reads them
    ref = grad.composite_vjp(planes, d, cam, d_out.astype(np.float32).astype(np.float64))
    _check(got, ref, f"d_planes {interp} {pdt}")


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
@pytest.mark.parametrize("kind", ["quilt3x2", "scattered"])
def test_composite_backward_2d_views(kind, interp):
    """Views with different vertical offsets: the row backward with views grouped by dy."""
    announce("composite backward 2d", kind, interp)
    cam = scenegen.camera(40, 36, 50.0, 3.0, math.radians(30.0), math.radians(10.0))
    g = geometry.derive(cam)
    K = 6
    p = scenegen.random_planes(K, g.hp, g.wp, seed=12)
    if kind == "quilt3x2":
        dx, dy, _, _ = geometry.quilt_views(cam, 3, 2)
    else:
        rng = np.random.default_rng(7)
        dy = np.array([0.03, -0.02, 0.03, 0.0, -0.02, 0.03, 0.05])
        dx = rng.uniform(-0.25, 0.25, len(dy))
    dx, dy = np.asarray(dx, np.float32), np.asarray(dy, np.float32)
    d = grad.composite_decisions(cam, p["depth"], dx, dy, interp)
    d_out = np.random.default_rng(3).normal(size=(len(dx), cam.ny, cam.nx, 4))
    got = host(T.composite_backward(ctx(), dev(p["rgba"]), dev(p["depth"]), cam, T.views_of(dx, dy),
                                    dev(d_out, torch.float32), interp))
    ref = grad.composite_vjp(np.asarray(p["rgba"], np.float32).astype(np.float64), d, cam,
                             d_out.astype(np.float32).astype(np.float64))
    _check(got, ref, f"d_planes 2d {kind} {interp}")


def _small_problem(seed=3, n=300, res=48, K=4, V=5, interp="nearest"):
    scene = scenegen.small_scene(n, seed)
    cam = scenegen.camera(res, res, 50.0, 3.0, math.radians(30.0))
    dx, dy = _views(cam, V)
    return scene, cam, K, dx, dy, interp


@pytest.mark.parametrize("seed", [3, 8])
def test_build_backward_matches_oracle(seed):
    """Random plane cotangents through lf_build_mpi_backward vs the oracle's VJP of the
    plane rasterisation (all parameters of all Gaussians)."""
    announce("build backward", seed)
    scene, cam, K, dx, dy, interp = _small_problem(seed)
    ds = T.to_device(scene)
    out = T.build_mpi(ctx(), ds, cam, K)
    rng = np.random.default_rng(seed)
    d_planes = rng.normal(size=tuple(out["rgba"].shape))
    gg = T.build_mpi_backward(ctx(), ds, cam, out, dev(d_planes, torch.float32))
    d = grad.decide(scene, cam, K, dx, dy, interp)
    ref = grad.planes_vjp(scene, cam, K, d, d_planes.astype(np.float32).astype(np.float64))
    for k in grad.KEYS:
        _check(host(gg[k]), ref[k], k)


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_lfrender_loss_gradient_matches_oracle_and_fd(interp):
    """End to end: L = sum (Q - Q*)^2 over views, pixels and RGB with Q* rendered from a
    perturbed copy; the LFRender gradient against the oracle gradient (all parameters) and
    against central differences of the oracle loss (64 parameters)."""
    announce("LFRender gradient", interp)
    scene, cam, K, dx, dy, _ = _small_problem(seed=5, interp=interp)
    target = scenegen.perturbed_target(scene, 6)
    td = T.to_device(target)
    views = T.views_of(dx, dy)
    with torch.no_grad():
        tout = T.build_mpi(ctx(), td, cam, K)
        timg = T.composite(ctx(), tout["rgba"], tout["depth"], cam, views, interp)
    params = {k: v.clone().requires_grad_(True) for k, v in T.to_device(scene).items() if k in grad.KEYS}
    img = T.render_light_field(ctx(), params, cam, views, K, interp)
    loss = ((img[..., :3] - timg[..., :3]) ** 2).sum()
    loss.backward()
    tgt = host(timg)
    rloss, rviews, rg, d = grad.loss_and_grad(scene, cam, K, dx, dy, tgt, interp)
    assert abs(float(loss) - rloss) <= 1e-4 * rloss
    for k in grad.KEYS:
        _check(host(params[k].grad), rg[k], k)
    # central differences of the frozen-decision FP64 loss
    rng = np.random.default_rng(7)
    vis = np.unique(d.gauss)
    tt = torch.as_tensor(tgt)
    for _ in range(64):
        key = grad.KEYS[rng.integers(0, 5)]
        i = int(rng.choice(vis))
        j = int(rng.integers(0, scene[key].shape[1])) if scene[key].ndim == 2 else None
        h = {"means": 1e-6, "log_scales": 1e-6, "quats": 1e-6, "opacity": 1e-7, "rgb": 1e-5}[key]
        vals = []
        for sgn in (1, -1):
            p = grad.params_of(scene, requires_grad=False)
            with torch.no_grad():
                if j is None:
                    p[key][i] += sgn * h
                else:
                    p[key][i, j] += sgn * h
            vals.append(float(grad.frozen_loss(p, cam, d, K, tt)[0]))
        fd = (vals[0] - vals[1]) / (2 * h)
        gk = host(params[key].grad)
        got = gk[i] if j is None else gk[i, j]
        scale = max(abs(fd), 1e-2 * np.abs(rg[key]).max())
        assert abs(got - fd) <= 1e-3 * scale, (key, i, j, got, fd)


def test_build_backward_culled_and_empty():
    announce("build backward culled/empty")
    scene = scenegen.small_scene(50, 1)
    scene["means"][:10, 2] = -3.0                      # behind the camera: culled, zero gradient
    cam = scenegen.camera(32, 32, 50.0, 3.0, math.radians(20.0))
    ds = T.to_device(scene)
    out = T.build_mpi(ctx(), ds, cam, 3)
    gg = T.build_mpi_backward(ctx(), ds, cam, out, torch.ones(tuple(out["rgba"].shape), device="cuda"))
    for k in grad.KEYS:
        a = host(gg[k])
        assert np.all(a[:10] == 0.0) and np.isfinite(a).all()
    assert np.abs(host(gg["rgb"])[10:]).max() > 0.0


def test_grad200k_full_size_sparse_cotangents():
    """The differentiation workload at full size (200,000 Gaussians, 512^2, 128 planes, 45
    views, FP32 planes): the composite backward for 300 random view pixels and the build
    backward for 40 covered plane texels, each against the oracle's local VJP (every
    texel / Gaussian compared; Gaussians whose inclusion or clamp decision at a chosen texel
    is within float32 rounding of its threshold are reported and skipped)."""
    from oracle import partition
    announce("grad200k full size")
    scene, cam, cfg = scenegen.config("grad200k")
    K = cfg["n_chunk"]
    ds = T.to_device(scene)
    ws = T.workspace_for(ds, cam, K)
    out = T.build_mpi(ctx(), ds, cam, K, workspace=ws)
    T.build_stats(ctx(), ws, check=True)
    g = geometry.derive(cam)
    part = partition.partition(scene["means"], cam, g, K)
    torch.cuda.synchronize()
    assert np.array_equal(out["chunk_of"].cpu().numpy(), part.chunk_of)
    dx, dy = _views(cam, cfg["vx"])
    views = T.views_of(dx, dy)
    rng = np.random.default_rng(12)
    # composite backward
    pix = np.unique(np.stack([rng.integers(0, len(dx), 300), rng.integers(0, cam.ny, 300),
                              rng.integers(0, cam.nx, 300)], 1), axis=0)
    cot = rng.normal(size=(pix.shape[0], 4))
    d_out = torch.zeros((len(dx), cam.ny, cam.nx, 4), dtype=torch.float32, device="cuda")
    d_out[tuple(torch.from_numpy(pix.T).cuda())] = torch.from_numpy(cot).float().cuda()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    dp = T.composite_backward(ctx(), out["rgba"], out["depth"], cam, views, d_out, "nearest")
    t1.record()
    torch.cuda.synchronize()
    print("composite backward ms", t0.elapsed_time(t1))
    planes32 = out["rgba"].cpu().numpy()
    ref = grad.pixel_vjp_sparse(lambda k, iy, ix: planes32[k, iy, ix].astype(np.float64), out["depth"].cpu().numpy(),
                                cam, dx, dy, "nearest", pix, cot.astype(np.float32).astype(np.float64))
    nz = torch.nonzero(dp.abs().sum(-1)).cpu().numpy()
    keys = list(ref.keys())
    assert {tuple(map(int, r)) for r in nz} <= set(keys)
    kk = np.array(keys)
    got = dp[tuple(torch.from_numpy(kk.T).cuda())].cpu().numpy()
    _check(got, np.stack([ref[k] for k in keys]), "d_planes (sparse, full size)")
    del dp, planes32
    # build backward
    alpha = out["rgba"][..., 3]
    cand = torch.nonzero(alpha > 0.05).cpu().numpy()
    tex = cand[rng.choice(cand.shape[0], 40, replace=False)]
    tcot = rng.normal(size=(tex.shape[0], 4)).astype(np.float32)
    dpl = torch.zeros(tuple(out["rgba"].shape), dtype=torch.float32, device="cuda")
    dpl[tuple(torch.from_numpy(tex.T).cuda())] = torch.from_numpy(tcot).cuda()
    t0.record()
    gg = T.build_mpi_backward(ctx(), ds, cam, out, dpl)
    t1.record()
    torch.cuda.synchronize()
    print("build backward ms", t0.elapsed_time(t1))
    amb = np.zeros(scene["means"].shape[0], dtype=bool)
    rg = grad.texel_vjp_local(scene, cam, part, tex, tcot.astype(np.float64), amb)
    print("Gaussians with a threshold-ambiguous decision:", int(amb.sum()))
    keep = ~amb
    touched = np.abs(rg["rgb"]).sum(1) > 0
    print("Gaussians touched:", int(touched.sum()))
    assert touched.sum() >= 40
    for k in grad.KEYS:
        _check(host(gg[k])[keep], rg[k][keep], k + " (full size)")


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_composite_backward_wide_windows(interp):
    """Planes just behind the reference camera magnify by 5-20 texels per pixel, so a
    work-group's window spans several LDS chunks; the chunked backward against the oracle."""
    announce("composite backward wide windows", interp)
    cam = scenegen.camera(200, 40, 50.0, 2.0, math.radians(40.0))
    g = geometry.derive(cam)
    K = 5
    p = scenegen.random_planes(K, g.hp, g.wp, seed=13, depth_range=(g.d_forward + 0.02, g.d_forward + 0.15))
    dx, dy = _views(cam, 12)
    d = grad.composite_decisions(cam, p["depth"], dx, dy, interp)
    d_out = np.random.default_rng(4).normal(size=(len(dx), cam.ny, cam.nx, 4))
    got = host(T.composite_backward(ctx(), dev(p["rgba"]), dev(p["depth"]), cam, T.views_of(dx, dy),
                                    dev(d_out, torch.float32), interp))
    ref = grad.composite_vjp(np.asarray(p["rgba"], np.float32).astype(np.float64), d, cam,
                             d_out.astype(np.float32).astype(np.float64))
    _check(got, ref, f"d_planes wide windows {interp}")


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
@pytest.mark.parametrize("group", [8, 12, 16])
@pytest.mark.parametrize("plane_scale", [1.0, 0.4])
def test_composite_backward_view_groups(plane_scale, group, interp, monkeypatch):
    """Every view-group size of the backward (LF_BWD_GROUP) with 20 views in two dy classes
    (groups cut short at each class end), for planes at the views' resolution (x -> texel
    slope about 0.6-1: lanes two apart never share a texel) and at 0.4 of it (slope about
    0.3: the phased update form)."""
    announce("composite backward view groups", plane_scale, group, interp)
    monkeypatch.setenv("LF_BWD_GROUP", str(group))
    cam = scenegen.camera(70, 20, 50.0, 3.0, math.radians(30.0), math.radians(8.0), plane_scale=plane_scale)
    g = geometry.derive(cam)
    K = 6
    p = scenegen.random_planes(K, g.hp, g.wp, seed=14)
    dx, dy, _, _ = geometry.quilt_views(cam, 10, 2)
    dx, dy = np.asarray(dx, np.float32), np.asarray(dy, np.float32)
    d = grad.composite_decisions(cam, p["depth"], dx, dy, interp)
    d_out = np.random.default_rng(5).normal(size=(len(dx), cam.ny, cam.nx, 4))
    got = host(T.composite_backward(ctx(), dev(p["rgba"]), dev(p["depth"]), cam, T.views_of(dx, dy),
                                    dev(d_out, torch.float32), interp))
    ref = grad.composite_vjp(np.asarray(p["rgba"], np.float32).astype(np.float64), d, cam,
                             d_out.astype(np.float32).astype(np.float64))
    _check(got, ref, f"d_planes groups of {group}, plane scale {plane_scale}, {interp}")
