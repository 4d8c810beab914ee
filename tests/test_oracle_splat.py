"""Pins of the oracle's EWA projection and plane rasterisation (Sec. 4.4): closed forms for
isotropic and axis-aligned Gaussians, a finite-difference Jacobian, scipy's rotation, the
two-Gaussian over operator and brute force over every texel of tiny scenes."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen
from oracle import geometry, partition, project, render, splat


def _one(means, log_scales, quat=(1.0, 0, 0, 0), opacity=0.8, rgb=(0.2, 0.5, 0.9)):
    n = len(means)
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return dict(means=f(means), log_scales=f(log_scales), quats=f([quat] * n),
                opacity=f([opacity] * n), rgb=f([rgb] * n))


CAM = scenegen.camera(96, 80, 50.0, 2.0, math.radians(30.0))
G = geometry.derive(CAM)


def test_quaternion_matches_scipy():
    q = np.random.default_rng(0).normal(size=(50, 4))
    R = project.quat_to_rot(q)
    Rs = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()       # scipy order: x, y, z, w
    assert np.allclose(R, Rs, atol=1e-13)


def test_isotropic_closed_form():
    """Sigma' = s^2 f'^2/Z^2 [[1+X^2/Z^2, XY/Z^2], [XY/Z^2, 1+Y^2/Z^2]] + f' I (f'_x = f'_y)."""
    cam = scenegen.camera(128, 128, 50.0, 2.0, math.radians(30.0))
    g = geometry.derive(cam)
    pts = [(0.3, -0.2, 3.0), (0.0, 0.0, 1.5), (-0.7, 0.4, 6.0)]
    s = 0.05
    sc = _one(pts, [[math.log(s)] * 3] * 3, quat=(0.3, -0.1, 0.7, 0.2))
    pr = project.project_reference(sc, np.arange(3), cam, g)
    f = g.fpx
    s = math.exp(float(sc["log_scales"][0, 0]))            # the float32-stored scale
    for i, (X, Y, zb) in enumerate(np.asarray(sc["means"], np.float64)):
        Z = zb - g.d_forward
        exp = s * s * f * f / (Z * Z) * np.array([[1 + X * X / Z / Z, X * Y / Z / Z], [X * Y / Z / Z, 1 + Y * Y / Z / Z]])
        exp += g.f_dilation * np.eye(2)
        assert np.allclose(pr.cov2d[i], exp, rtol=1e-12)
        assert pr.mean2d[i] == pytest.approx([f * X / Z + g.cpx, f * Y / Z + g.cpy], rel=1e-14)
        assert np.linalg.det(pr.cov2d[i]) >= g.f_dilation ** 2


def test_axis_aligned_and_quaternion_order():
    """On axis, an axis-aligned Gaussian projects to diag(f^2 s_x^2/Z^2, f^2 s_y^2/Z^2) + f' I;
    a 90-degree turn about z (w = cos 45, z = sin 45) swaps the two axes."""
    sx, sy, sz = 0.02, 0.07, 0.04
    Z = 3.0
    sc = _one([(0, 0, Z + G.d_forward)], [[math.log(sx), math.log(sy), math.log(sz)]])
    pr = project.project_reference(sc, [0], CAM, G)
    assert np.allclose(pr.cov2d[0], np.diag([(G.fpx * sx / Z) ** 2, (G.fpy * sy / Z) ** 2]) + G.f_dilation * np.eye(2), rtol=1e-6)
    h = math.sqrt(0.5)
    sc = _one([(0, 0, Z + G.d_forward)], [[math.log(sx), math.log(sy), math.log(sz)]], quat=(h, 0, 0, h))
    pr = project.project_reference(sc, [0], CAM, G)
    assert np.allclose(pr.cov2d[0], np.diag([(G.fpx * sy / Z) ** 2, (G.fpy * sx / Z) ** 2]) + G.f_dilation * np.eye(2), rtol=1e-6)


def test_jacobian_is_derivative_of_projection():
    """J of the EWA step equals the finite-difference derivative of p -> (f x/z + c, f y/z + c);
    Sigma' - f'I then equals J Sigma J^T recovered from columns of unit-covariance Gaussians."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        p = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(1.5, 6)])
        h = 1e-6

        def proj(q):
            z = q[2] - G.d_forward
            return np.array([G.fpx * q[0] / z + G.cpx, G.fpy * q[1] / z + G.cpy])
        Jfd = np.stack([(proj(p + h * e) - proj(p - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        # a Gaussian with covariance e_i e_i^T (+ tiny isotropic) isolates column i of J
        s = 1e-3
        sc = _one([p], [[math.log(s)] * 3])
        pr = project.project_reference(sc, [0], CAM, G)
        iso = s * s * Jfd @ Jfd.T + G.f_dilation * np.eye(2)
        assert np.allclose(pr.cov2d[0], iso, rtol=1e-6)


def test_single_gaussian_plane_closed_form():
    """A lone on-axis isotropic Gaussian: texel = (alpha rgb, alpha), alpha = min(0.99, o exp(-r^2/2 sigma^2))
    where o exp(...) >= 1/255, with sigma^2 = (s f'/Z)^2 + f'."""
    cam = scenegen.camera(40, 40, 50.0, 2.0, math.radians(30.0))
    g = geometry.derive(cam)
    for o in (0.3, 0.999):
        s, Z = 0.03, 2.0
        sc = _one([(0, 0, Z + g.d_forward)], [[math.log(s)] * 3], opacity=o, rgb=(0.25, 0.5, 1.0))
        pr = project.project_reference(sc, [0], cam, g)
        rgba, amb = splat.render_plane(pr, g.hp, g.wp)
        s = math.exp(float(sc["log_scales"][0, 0]))
        Z = float(sc["means"][0, 2]) - g.d_forward
        sig2 = (s * g.fpx / Z) ** 2 + g.f_dilation
        oo = float(np.float32(o))
        for j in range(g.hp):
            for i in range(g.wp):
                r2 = (i - g.cpx) ** 2 + (j - g.cpy) ** 2
                a = oo * math.exp(-r2 / (2 * sig2))
                al = min(0.99, a) if a >= 1 / 255 else 0.0
                assert rgba[j, i] == pytest.approx([al * 0.25, al * 0.5, al * 1.0, al], abs=1e-12)
        assert (rgba[..., 3] > 0).sum() >= 9 and not amb.all()


def test_two_gaussian_over_operator():
    """Front Gaussian first: C = a1 c1 + (1 - a1) a2 c2, A = 1 - (1 - a1)(1 - a2)."""
    cam = scenegen.camera(32, 32, 50.0, 2.0, math.radians(20.0))
    g = geometry.derive(cam)
    sc = _one([(0, 0, 2.5), (0, 0, 3.5)], [[math.log(0.05)] * 3] * 2, opacity=0.7)
    sc["rgb"][1] = [0.9, 0.1, 0.4]
    sc["opacity"][1] = 0.6
    p = partition.partition(sc["means"], cam, g, 1, "quantile")
    assert p.order.tolist() == [0, 1]
    pr = project.project_reference(sc, p.order, cam, g)
    rgba, _ = splat.render_plane(pr, g.hp, g.wp)
    j = i = 16
    a = []
    for n in range(2):
        d = np.array([i, j]) - pr.mean2d[n]
        an = pr.opacity[n] * math.exp(-0.5 * d @ pr.conic[n] @ d)
        a.append(min(0.99, an))
    c1, c2 = pr.rgb[0], pr.rgb[1]
    assert rgba[j, i, :3] == pytest.approx(a[0] * c1 + (1 - a[0]) * a[1] * c2, abs=1e-12)
    assert rgba[j, i, 3] == pytest.approx(1 - (1 - a[0]) * (1 - a[1]), abs=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plane_brute_force(seed):
    """Every texel by plain loops over the chunk's Gaussians in sorted order, no bounding boxes."""
    cam = scenegen.camera(24, 20, 50.0, 2.0, math.radians(35.0))
    g = geometry.derive(cam)
    sc = scenegen.small_scene(12, seed)
    K = 3
    mpi = render.build_mpi_gaussians(sc, cam, K)
    order = sorted((float(mpi.part.key[i]), i) for i in range(12) if mpi.part.visible[i])
    for k in range(K):
        members = [i for r, (_, i) in enumerate(order) if (r * K) // len(order) == k]
        pr = project.project_reference(sc, members, cam, g)
        for j in range(g.hp):
            for i in range(g.wp):
                C = np.zeros(3)
                T = 1.0
                for n in range(len(members)):
                    d = np.array([i, j], float) - pr.mean2d[n]
                    a = pr.opacity[n] * math.exp(-0.5 * d @ pr.conic[n] @ d)
                    if a >= 1 / 255:
                        al = min(0.99, a)
                        C += al * T * pr.rgb[n]
                        T *= 1 - al
                assert np.allclose(mpi.planes[k, j, i], [*C, 1 - T], atol=1e-12)
        # the vectorised per-texel path agrees with the per-Gaussian path
        jj, ii = np.mgrid[0:g.hp, 0:g.wp]
        v, a = splat.blend_texels(pr, ii.ravel(), jj.ravel())
        assert np.allclose(v.reshape(g.hp, g.wp, 4), mpi.planes[k], atol=1e-12)
        assert np.array_equal(a.reshape(g.hp, g.wp), mpi.ambiguous[k])


def test_ambiguity_flags_threshold_texels():
    """A texel whose footprint value sits on 1/255 is flagged; the flag band is narrow."""
    cam = scenegen.camera(64, 64, 50.0, 2.0, math.radians(30.0))
    g = geometry.derive(cam)
    sc = _one([(0, 0, 3.0)], [[math.log(0.05)] * 3], opacity=0.5)
    pr = project.project_reference(sc, [0], cam, g)
    sig2 = pr.cov2d[0, 0, 0]
    r_edge = math.sqrt(2 * sig2 * math.log(255 * pr.opacity[0]))
    # texels exactly at distance r_edge from the mean (shift the mean so one lands there)
    pr.mean2d[0] = [10.0 - r_edge, 20.0]
    rgba, amb = splat.render_plane(pr, g.hp, g.wp)
    assert amb[20, 10] and amb.sum() <= 3


@pytest.mark.parametrize("seed", [0, 3])
def test_support_pairs_brute_force(seed):
    """support_pairs against plain loops over every texel of the plane and every Gaussian
    (o G >= 1/255, no bounding boxes)."""
    cam = scenegen.camera(40, 32, 50.0, 2.0, math.radians(35.0))
    g = geometry.derive(cam)
    sc = scenegen.small_scene(30, seed)
    K = 3
    part = partition.partition(sc["means"], cam, g, K, "quantile", None)
    for k in range(K):
        pr = render.chunk_projection(sc, cam, g, part, k)
        got, near = splat.support_pairs(pr, g.hp, g.wp)
        want = 0
        for n in range(pr.mean2d.shape[0]):
            for j in range(g.hp):
                for i in range(g.wp):
                    d = np.array([i, j], float) - pr.mean2d[n]
                    want += pr.opacity[n] * math.exp(-0.5 * d @ pr.conic[n] @ d) >= 1.0 / 255.0
        assert got == want and near <= got + 10
