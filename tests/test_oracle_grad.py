"""Pins of the gradient oracle: its torch forward is the numpy oracle's forward, its
autograd gradient equals central finite differences of the frozen-decision loss, and a
one-Gaussian case has a closed form."""
import math

import numpy as np
import pytest
import torch

import scenegen
from oracle import composite, geometry, grad, render


def _setup(n=40, seed=3, res=24, K=3, views=3, interp="nearest", phi=20.0):
    scene = scenegen.small_scene(n, seed)
    cam = scenegen.camera(res, res, 50.0, 3.0, math.radians(phi))
    dx, dy, _, _ = geometry.quilt_views(cam, views, 1)
    return scene, cam, K, dx.astype(np.float32), dy.astype(np.float32), interp


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_torch_forward_is_the_oracle_forward(interp):
    scene, cam, K, dx, dy, _ = _setup(interp=interp)
    d = grad.decide(scene, cam, K, dx, dy, interp)
    p = grad.params_of(scene, requires_grad=False)
    planes = grad.planes_of(p, cam, d, K).numpy()
    mpi = render.build_mpi_gaussians(scene, cam, K)
    np.testing.assert_allclose(planes, mpi.planes, atol=1e-12)
    assert planes[..., 3].max() > 0.5
    views = grad.composite_of(torch.from_numpy(planes), d, cam).numpy()
    ref, _ = composite.composite(mpi.planes, mpi.depth, cam, mpi.geom, dx, dy, interp)
    np.testing.assert_allclose(views, ref, atol=1e-12)


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_autograd_matches_central_differences(interp):
    """Central differences (a step scaled for float64) of the
    loss with frozen decisions against the autograd gradient on 40 random parameters."""
    scene, cam, K, dx, dy, _ = _setup(interp=interp)
    target = scenegen.perturbed_target(scene, 9)
    d = grad.decide(scene, cam, K, dx, dy, interp)
    tgt_views = grad.composite_of(grad.planes_of(grad.params_of(target, False), cam, grad.decide(target, cam, K, dx, dy, interp), K),
                                  grad.decide(target, cam, K, dx, dy, interp), cam).detach()
    loss, views, g, _ = grad.loss_and_grad(scene, cam, K, dx, dy, tgt_views, interp, d)
    assert loss > 0
    rng = np.random.default_rng(1)
    vis = np.unique(d.gauss)
    checked = 0
    for _ in range(40):
        key = grad.KEYS[rng.integers(0, 5)]
        i = int(rng.choice(vis))
        j = int(rng.integers(0, scene[key].shape[1])) if scene[key].ndim == 2 else None
        h = {"means": 1e-6, "log_scales": 1e-6, "quats": 1e-6, "opacity": 1e-7, "rgb": 1e-5}[key]
        vals = []
        for s in (+1, -1):
            p = grad.params_of(scene, requires_grad=False)
            with torch.no_grad():
                if j is None:
                    p[key][i] += s * h
                else:
                    p[key][i, j] += s * h
            vals.append(float(grad.frozen_loss(p, cam, d, K, tgt_views)[0]))
        fd = (vals[0] - vals[1]) / (2 * h)
        ad = g[key][i] if j is None else g[key][i, j]
        scale = max(abs(ad), 1e-3 * np.abs(g[key]).max())
        assert abs(fd - ad) <= 1e-5 * scale + 1e-9, (key, i, j, fd, ad)
        checked += 1
    assert checked == 40


def test_single_gaussian_colour_gradient_closed_form():
    """One Gaussian, one plane, one view at zero baseline: Q = alpha rgb per pixel, so
    dL/drgb = sum_pixels 2 (Q - Q*) alpha."""
    scene = scenegen.small_scene(1, 4)
    scene["means"][0] = [0.0, 0.0, 3.0]
    scene["log_scales"][0] = [-2.0, -2.2, -2.1]
    cam = scenegen.camera(17, 17, 50.0, 3.0, 0.0)
    dx = np.zeros(1, np.float32)
    d = grad.decide(scene, cam, 1, dx, dx)
    target = torch.zeros(1, 17, 17, 4, dtype=torch.float64)
    loss, views, g, _ = grad.loss_and_grad(scene, cam, 1, dx, dx, target, "nearest", d)
    alpha = 1.0 - views[0, ..., 3]
    expect = (2.0 * views[0, ..., :3] * alpha[..., None]).sum(axis=(0, 1))
    np.testing.assert_allclose(g["rgb"][0], expect, rtol=1e-12)
    np.testing.assert_allclose(views[0, ..., :3], alpha[..., None] * scene["rgb"][0].astype(np.float64), rtol=1e-12)


def test_vjps_compose_to_the_loss_gradient():
    scene, cam, K, dx, dy, interp = _setup(seed=5)
    d = grad.decide(scene, cam, K, dx, dy, interp)
    target = torch.zeros(len(dx), cam.ny, cam.nx, 4, dtype=torch.float64)
    loss, views, g, _ = grad.loss_and_grad(scene, cam, K, dx, dy, target, interp, d)
    p = grad.params_of(scene, requires_grad=False)
    planes = grad.planes_of(p, cam, d, K).numpy()
    d_out = np.zeros_like(views)
    d_out[..., :3] = 2.0 * views[..., :3]
    d_planes = grad.composite_vjp(planes, d, cam, d_out)
    g2 = grad.planes_vjp(scene, cam, K, d, d_planes)
    for k in grad.KEYS:
        np.testing.assert_allclose(g2[k], g[k], rtol=1e-10, atol=1e-12)


def test_composite_vjp_matches_finite_differences_on_planes():
    """The composite's plane gradient, including the alpha term -T_k (g . R_{k+1} + g_T S_{k+1})
    with a transmittance cotangent, against central differences on random texels."""
    scene, cam, K, dx, dy, _ = _setup(seed=6)
    d = grad.decide(scene, cam, K, dx, dy, "bilinear")
    planes = scenegen.random_planes(K, cam.ny, cam.nx, seed=2)["rgba"].astype(np.float64)
    rng = np.random.default_rng(4)
    d_out = rng.normal(size=(len(dx), cam.ny, cam.nx, 4))
    gp = grad.composite_vjp(planes, d, cam, d_out)

    def f(pl):
        return float((grad.composite_of(torch.from_numpy(pl), d, cam).numpy() * d_out).sum())
    for _ in range(30):
        k, y, x, c = rng.integers(0, K), rng.integers(0, cam.ny), rng.integers(0, cam.nx), rng.integers(0, 4)
        e = np.zeros_like(planes)
        e[k, y, x, c] = 1e-6
        fd = (f(planes + e) - f(planes - e)) / 2e-6
        assert abs(fd - gp[k, y, x, c]) <= 1e-6 * max(1.0, abs(fd))


def test_local_vjps_match_the_dense_oracle():
    """The footprint-local texel VJP and the sparse pixel VJP (used at full size) equal the
    dense oracle VJPs on a small problem."""
    scene, cam, K, dx, dy, _ = _setup(seed=7, n=60)
    for interp in ("nearest", "bilinear"):
        d = grad.decide(scene, cam, K, dx, dy, interp)
        rng = np.random.default_rng(3)
        g = d.geom
        tex = np.stack([rng.integers(0, K, 12), rng.integers(0, g.hp, 12), rng.integers(0, g.wp, 12)], 1)
        tex = np.unique(tex, axis=0)
        cot = rng.normal(size=(tex.shape[0], 4))
        dense = np.zeros((K, g.hp, g.wp, 4))
        dense[tex[:, 0], tex[:, 1], tex[:, 2]] = cot
        ref = grad.planes_vjp(scene, cam, K, d, dense)
        got = grad.texel_vjp_local(scene, cam, d.part, tex, cot)
        for k in grad.KEYS:
            np.testing.assert_allclose(got[k], ref[k], rtol=1e-9, atol=1e-12)
        planes = grad.planes_of(grad.params_of(scene, False), cam, d, K).numpy()
        pix = np.stack([rng.integers(0, len(dx), 15), rng.integers(0, cam.ny, 15), rng.integers(0, cam.nx, 15)], 1)
        pix = np.unique(pix, axis=0)
        pc = rng.normal(size=(pix.shape[0], 4))
        d_out = np.zeros((len(dx), cam.ny, cam.nx, 4))
        d_out[pix[:, 0], pix[:, 1], pix[:, 2]] = pc
        dref = grad.composite_vjp(planes, d, cam, d_out)
        sp = grad.pixel_vjp_sparse(lambda k, iy, ix: planes[k, iy, ix], d.part.depth, cam, dx, dy, interp, pix, pc)
        dsp = np.zeros_like(dref)
        for (k, y, x), v in sp.items():
            dsp[k, y, x] = v
        np.testing.assert_allclose(dsp, dref, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_footprint_fd_equals_whole_frame_fd(interp):
    """The footprint-local central difference (the Gaussian's frozen support in its plane and
    the pixels that reach it) equals the central difference of the whole frozen-decision
    loss over every pixel of every view, on 30 random (Gaussian, parameter) pairs with the
    full-size steps (1e-4 means / log-scales / quaternions, 1e-5 opacity, 1e-3 colour)."""
    scene, cam, K, dx, dy, _ = _setup(n=60, seed=4, res=32, K=3, views=4, interp=interp)
    target = composite.composite(render.build_mpi_gaussians(scenegen.perturbed_target(scene, 2), cam, K).planes,
                                 render.build_mpi_gaussians(scene, cam, K).depth, cam, geometry.derive(cam), dx, dy,
                                 interp)[0]
    d = grad.decide(scene, cam, K, dx, dy, interp)
    mpi = render.build_mpi_gaussians(scene, cam, K)
    tt = torch.as_tensor(target)
    rng = np.random.default_rng(5)
    vis = np.unique(d.gauss)
    steps = {"means": 1e-4, "log_scales": 1e-4, "quats": 1e-4, "opacity": 1e-5, "rgb": 1e-3}
    checked = 0
    for _ in range(30):
        key = grad.KEYS[rng.integers(0, 5)]
        i = int(rng.choice(vis))
        j = int(rng.integers(0, scene[key].shape[1])) if scene[key].ndim == 2 else None
        h = steps[key]
        local, amb, support = grad.footprint_fd(scene, cam, d.part, mpi.planes, dx, dy, target, i, key, j, h, interp)
        vals = []
        for sgn in (1, -1):
            p = grad.params_of(scene, requires_grad=False)
            with torch.no_grad():
                if j is None:
                    p[key][i] += sgn * h
                else:
                    p[key][i, j] += sgn * h
            vals.append(float(grad.frozen_loss(p, cam, d, K, tt)[0]))
        whole = (vals[0] - vals[1]) / (2 * h)
        assert abs(local - whole) <= 1e-7 * max(abs(whole), 1e-3), (key, i, j, local, whole)
        checked += abs(whole) > 1e-6
        assert support or whole == 0.0
    assert checked >= 20
