"""Host-side checks of the C ABI (no GPU): the library loads and exports every declared
symbol, host geometry matches the oracle bit for bit after float32 rounding, and invalid
arguments are rejected before any device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import scenegen
from oracle import decisions, geometry

L = pytest.importorskip("paper_2508_18540_amd._lib")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("liblf.so is not built (run __graft_entry__.build())")
    return L.load()


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "lf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(L.EXPORTS)
    assert "gfx950" in L.lf_version()


CAMS = {
    "uniform10k": scenegen.config_camera("uniform10k")[0],
    "cluster500k": scenegen.config_camera("cluster500k")[0],
    "voxel256": scenegen.config_camera("voxel256")[0],
    "shifted": scenegen.camera(300, 200, 60.0, 1.5, math.radians(25.0), math.radians(10.0), plane_scale=1.5,
                               d_shift=0.2, z_near=0.1),
    "rotated": scenegen.camera(128, 96, 45.0, 3.0, math.radians(35.0), R=[[0, 0, 1], [0, 1, 0], [-1, 0, 0]],
                               t=[0.5, -0.25, 4.0]),
    "constant_filter": scenegen.camera(160, 120, 50.0, 2.0, math.radians(30.0), plane_scale=2.0, dilation=0.3),
}


@pytest.mark.parametrize("name", sorted(CAMS))
def test_host_geometry_bit_exact(lib, name):
    cam = CAMS[name]
    info = L.lf_geometry(L.make_camera(cam))
    g = geometry.derive(cam)
    c = decisions.constants(g, cam)
    assert info.d_forward0 == pytest.approx(g.d_forward0, rel=1e-15, abs=1e-300)
    assert info.tan_half_theta_prime_x == pytest.approx(g.tpx, rel=1e-15)
    assert info.f_dilation == pytest.approx(g.f_dilation, rel=1e-15)
    assert (info.plane_width, info.plane_height) == (g.wp, g.hp)
    pairs = [("d_forward32", c.d_forward), ("guard_x32", c.guard_x), ("guard_y32", c.guard_y),
             ("ratio_x32", c.ratio_x), ("ratio_y32", c.ratio_y), ("fpx32", c.fpx), ("fpy32", c.fpy),
             ("cpx32", c.cpx), ("cpy32", c.cpy), ("cx32", c.cx), ("cy32", c.cy), ("inv_focal32", c.inv_focal)]
    for field, ref in pairs:
        got = np.float32(getattr(info, field))
        assert got.view(np.uint32) == np.float32(ref).view(np.uint32), field


@pytest.mark.parametrize("vx,vy", [(9, 1), (45, 1), (1, 1), (5, 3)])
def test_quilt_views_match_eq3_eq4(lib, vx, vy):
    cam = CAMS["shifted"]
    v = L.lf_quilt_views(L.make_camera(cam), vx, vy)
    dx, dy, _, _ = geometry.quilt_views(cam, vx, vy)
    got = np.array([[e.dx, e.dy] for e in v], dtype=np.float32)
    assert np.array_equal(got[:, 0].view(np.uint32), dx.astype(np.float32).view(np.uint32))
    assert np.array_equal(got[:, 1].view(np.uint32), dy.astype(np.float32).view(np.uint32))


def _valid_call(lib, **kw):
    cam = L.make_camera(CAMS["uniform10k"])
    for k, v in kw.pop("cam", {}).items():
        setattr(cam, k, v)
    mpi = L.make_mpi(kw.pop("dtype", L.LF_F32), kw.pop("n_chunk", 16), kw.pop("h", 128), kw.pop("w", 128),
                     kw.pop("rgba", 0x1000), kw.pop("depth", 0x2000))
    views = L.make_views([0.0, 0.01], [0.0, 0.0])
    n_views = kw.pop("n_views", 2)
    st = lib.lf_composite(kw.pop("ctx", None), ctypes.byref(mpi), ctypes.byref(cam), views, n_views,
                          kw.pop("interp", 0), kw.pop("out_dtype", 0), kw.pop("out", 0x3000), None)
    return st, L.lf_last_error()


@pytest.mark.parametrize("kw,needle", [
    (dict(cam=dict(nx=0)), "resolution"),
    (dict(cam=dict(fov_x=math.pi)), "field of view"),
    (dict(cam=dict(d_focal=-1.0)), "d_focal"),
    (dict(cam=dict(phi_x=-0.1)), "viewing angles"),
    (dict(cam=dict(z_near=0.0)), "z_near"),
    (dict(cam=dict(plane_scale=float("nan"))), "plane_scale"),
    (dict(cam=dict(dilation=-0.1)), "dilation"),
    (dict(cam=dict(dilation=float("inf"))), "dilation"),
    (dict(dtype=7), "dtype"),
    (dict(n_chunk=0), "n_chunk"),
    (dict(w=64), "planes are"),
    (dict(rgba=0), "rgba"),
    (dict(n_views=0), "n_views"),
    (dict(n_views=300), "n_views"),
    (dict(interp=5), "interp"),
    (dict(out_dtype=2), "out_dtype"),
    (dict(out=0), "out is NULL"),
    (dict(), "ctx is NULL"),
])
def test_composite_rejects_invalid_arguments(lib, kw, needle):
    st, msg = _valid_call(lib, **kw)
    assert st == L.LF_ERR_INVALID_ARG
    assert needle in msg


def test_geometry_rejects_null(lib):
    assert lib.lf_geometry(None, None) == L.LF_ERR_INVALID_ARG
    assert lib.lf_quilt_views(ctypes.byref(L.make_camera(CAMS["uniform10k"])), 0, 1,
                              (L.lf_view * 1)()) == L.LF_ERR_INVALID_ARG


def _field(kind, n=10, **kw):
    f = L.lf_field()
    f.kind, f.n = kind, n
    if kind == L.LF_GAUSSIANS:
        f.means, f.log_scales, f.quats, f.opacity, f.rgb = 0x1000, 0x2000, 0x3000, 0x4000, 0x5000
    else:
        f.ijk, f.density, f.rgb = 0x1000, 0x2000, 0x3000
        f.origin[:] = [-1.0, -1.0, 3.0]
        f.voxel_size = 2.0 / 256
    for k, v in kw.items():
        if k == "origin":
            f.origin[:] = v
        else:
            setattr(f, k, v)
    return f


@pytest.mark.parametrize("kind,kw,needle", [
    (L.LF_GAUSSIANS, dict(means=0), "Gaussian attribute"),
    (L.LF_GAUSSIANS, dict(n=-1), "field size"),
    (L.LF_GAUSSIANS, dict(n=1 << 28), "field size"),
    (L.LF_VOXELS, dict(density=0), "voxel attribute"),
    (L.LF_VOXELS, dict(voxel_size=0.0), "voxel_size"),
    (L.LF_VOXELS, dict(voxel_size=float("inf")), "voxel_size"),
    (L.LF_VOXELS, dict(origin=[0.0, float("nan"), 0.0]), "origin"),
    (7, dict(), "field kind"),
])
def test_build_rejects_invalid_fields(lib, kind, kw, needle):
    cam = L.make_camera(CAMS["uniform10k"])
    f = _field(kind, **kw)
    nbytes = ctypes.c_size_t(0)
    st = lib.lf_build_mpi_workspace(ctypes.byref(f), ctypes.byref(cam), 16, 0, ctypes.byref(nbytes))
    assert st == L.LF_ERR_INVALID_ARG
    assert needle in L.lf_last_error()


@pytest.mark.parametrize("kind", [L.LF_GAUSSIANS, L.LF_VOXELS])
def test_build_workspace_size_and_capacity_errors(lib, kind):
    cam = L.make_camera(CAMS["uniform10k"])
    f = _field(kind, n=10_000)
    nbytes = ctypes.c_size_t(0)
    assert lib.lf_build_mpi_workspace(ctypes.byref(f), ctypes.byref(cam), 16, 0, ctypes.byref(nbytes)) == L.LF_OK
    assert nbytes.value > 10_000 * 64
    big = ctypes.c_size_t(0)
    assert lib.lf_build_mpi_workspace(ctypes.byref(f), ctypes.byref(cam), 16, 4_000_000, ctypes.byref(big)) == L.LF_OK
    assert big.value > nbytes.value
    # too small a workspace is a capacity error, reported before anything is enqueued
    mpi = L.make_mpi(L.LF_F32, 16, 128, 128, 0x6000, 0x7000)
    st = lib.lf_build_mpi(None, ctypes.byref(f), ctypes.byref(cam), 16, 0, None, ctypes.byref(mpi), 0x8000, 1024,
                          None)
    assert st == L.LF_ERR_CAPACITY
    assert "too small" in L.lf_last_error()
    # inverse-depth binning needs a range beyond D_forward
    st = lib.lf_build_mpi(None, ctypes.byref(f), ctypes.byref(cam), 16, 1, None, ctypes.byref(mpi), 0x8000,
                          nbytes.value, None)
    assert st == L.LF_ERR_INVALID_ARG


def test_batch_rejects_invalid_items(lib):
    cam = L.make_camera(CAMS["uniform10k"])
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)                 # never dereferenced: validation fails first
    assert lib.lf_batch_create(dummy, None, 1, 0, ctypes.byref(h)) == L.LF_ERR_INVALID_ARG
    it = L.lf_batch_item()
    it.field = _field(L.LF_GAUSSIANS)
    it.cam = cam
    it.n_chunk = 16
    it.views = L.make_views([0.0], [0.0])
    it.n_views = 1
    it.mpi = L.make_mpi(L.LF_F32, 16, 128, 128, 0x6000, 0x7000)
    it.out, it.workspace, it.workspace_bytes = 0x9000, 0x8000, 1 << 30
    arr = (L.lf_batch_item * 1)(it)
    assert lib.lf_batch_create(dummy, arr, 0, 0, ctypes.byref(h)) == L.LF_ERR_INVALID_ARG
    assert lib.lf_batch_create(dummy, arr, 1, 8, ctypes.byref(h)) == L.LF_ERR_INVALID_ARG
    for field, value, needle in [("interp", 3, "interp"), ("out_dtype", 5, "out_dtype"), ("binning", 4, "binning"),
                                 ("n_views", 0, "n_views"), ("out", 0, "NULL")]:
        bad = L.lf_batch_item.from_buffer_copy(it)
        setattr(bad, field, value)
        st = lib.lf_batch_create(dummy, (L.lf_batch_item * 1)(bad), 1, 0, ctypes.byref(h))
        assert st == L.LF_ERR_INVALID_ARG, field
        assert needle in L.lf_last_error(), (field, L.lf_last_error())


def test_render_view_rejects_invalid_arguments(lib):
    """The per-view render validates everything on the host before touching the device."""
    cam = L.make_camera(CAMS["uniform10k"])
    g = L.lf_geometry(cam)
    f = _field(L.LF_GAUSSIANS, n=1000)
    nbytes = ctypes.c_size_t(0)
    assert lib.lf_render_view_workspace(ctypes.byref(f), ctypes.byref(cam), ctypes.byref(nbytes)) == L.LF_OK
    one = ctypes.c_size_t(0)
    assert lib.lf_build_mpi_workspace(ctypes.byref(f), ctypes.byref(cam), 1, 0, ctypes.byref(one)) == L.LF_OK
    assert 0 < nbytes.value <= one.value              # one plane at the view size (P_s = 1)
    v = L.lf_view(0.1, 0.0)
    ok = L.make_mpi(L.LF_F32, 1, cam.ny, cam.nx, 0x6000, 0x7000)
    cases = [
        (dict(view=None), "view"),
        (dict(view=L.lf_view(float("nan"), 0.0)), "not finite"),
        (dict(out=L.make_mpi(L.LF_F32, 2, cam.ny, cam.nx, 0x6000, 0x7000)), "one"),
        (dict(out=L.make_mpi(L.LF_F32, 1, g.plane_height + 8, g.plane_width, 0x6000, 0x7000)), "one"),
        (dict(out=L.make_mpi(9, 1, cam.ny, cam.nx, 0x6000, 0x7000)), "dtype"),
        (dict(nbytes=1024), "too small"),
        (dict(field=_field(L.LF_VOXELS, n=1000)), "Gaussian fields only"),
    ]
    for kw, needle in cases:
        fld = kw.get("field", f)
        view = kw.get("view", v)
        out = kw.get("out", ok)
        st = lib.lf_render_view(None, ctypes.byref(fld), ctypes.byref(cam), ctypes.byref(view) if view else None,
                                ctypes.byref(out), 0x8000, kw.get("nbytes", nbytes.value), None)
        assert st != L.LF_OK, kw
        assert needle in L.lf_last_error(), (kw, L.lf_last_error())


def test_sh_entry_points_reject_invalid_arguments(lib):
    """The SH build, composite and colour entry points validate on the host first."""
    assert [lib.lf_sh_texel_floats(d) for d in (-1, 0, 1, 2, 3, 4)] == [0, 4, 16, 28, 52, 0]
    cam = L.make_camera(CAMS["uniform10k"])
    g = L.lf_geometry(cam)
    f = _field(L.LF_GAUSSIANS, n=1000)
    nbytes = ctypes.c_size_t(0)
    assert lib.lf_build_mpi_workspace(ctypes.byref(f), ctypes.byref(cam), 4, 0, ctypes.byref(nbytes)) == L.LF_OK

    def sh_mpi(degree=2, K=4, h=g.plane_height, w=g.plane_width):
        return L.lf_sh_mpi(degree, K, h, w, 0x6000, 0x7000)

    build_cases = [
        (dict(mpi=sh_mpi(degree=4)), "degree"),
        (dict(mpi=sh_mpi(K=3)), "n_chunk"),
        (dict(mpi=sh_mpi(h=g.plane_height + 2)), "planes are"),
        (dict(sh=None), "sh is NULL"),
        (dict(field=_field(L.LF_VOXELS, n=1000)), "Gaussian fields only"),
        (dict(nbytes=1024), "too small"),
    ]
    for kw, needle in build_cases:
        m = kw.get("mpi", sh_mpi())
        st = lib.lf_build_mpi_sh(None, ctypes.byref(kw.get("field", f)), kw.get("sh", 0x9000), ctypes.byref(cam), 4,
                                 L.LF_BIN_QUANTILE, None, ctypes.byref(m), 0x8000, kw.get("nbytes", nbytes.value), None)
        assert st != L.LF_OK, kw
        assert needle in L.lf_last_error(), (kw, L.lf_last_error())
    views = L.make_views([0.0, 0.1], [0.0, 0.0])
    comp_cases = [
        (dict(mpi=sh_mpi(degree=-1)), "degree"),
        (dict(interp=7), "interp"),
        (dict(out=None), "out is NULL"),
        (dict(mpi=sh_mpi(w=g.plane_width + 1)), "planes are"),
        (dict(n_views=0), "n_views"),
    ]
    for kw, needle in comp_cases:
        m = kw.get("mpi", sh_mpi())
        st = lib.lf_composite_sh(None, ctypes.byref(m), ctypes.byref(cam), views, kw.get("n_views", 2),
                                 kw.get("interp", L.LF_NEAREST), kw.get("out", 0xa000), None)
        assert st != L.LF_OK, kw
        assert needle in L.lf_last_error(), (kw, L.lf_last_error())
    v = L.lf_view(0.0, 0.0)
    colour_cases = [
        (dict(degree=4), "degree"),
        (dict(n=-1), "negative"),
        (dict(means=None), "NULL"),
        (dict(view=L.lf_view(float("inf"), 0.0)), "not finite"),
    ]
    for kw, needle in colour_cases:
        st = lib.lf_sh_colours(None, kw.get("means", 0x1000), 0x2000, kw.get("degree", 1), kw.get("n", 10),
                               ctypes.byref(cam), ctypes.byref(kw.get("view", v)), 0x3000, None)
        assert st != L.LF_OK, kw
        assert needle in L.lf_last_error(), (kw, L.lf_last_error())
