"""GPU parity of the Gaussian MPI build (lf_build_mpi; Sec. 4.4, Alg. 1 steps 1-5) and of
the whole frame (build + composite) against the FP64 oracle.

Chunk indices, chunk counts and plane depths must match bit for bit.  Plane texels and
composited pixels must match to 1e-4 except where the oracle flags the 1/255 inclusion
threshold as ambiguous (both outcomes correct); those must stay within the jump one
threshold Gaussian can cause."""
import math

import numpy as np
import pytest
import torch

import scenegen
from oracle import composite, geometry, partition, project, quantize, render, splat
from paper_2508_18540_amd import _lib as L
from paper_2508_18540_amd import torch_api as T
from tests.gpu_util import announce, ctx, host, psnr

pytestmark = pytest.mark.gpu

TDT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def _gpu_build(scene, cam, K, binning="quantile", rng=None, dtype=torch.float32, cap=0):
    ds = T.to_device(scene)
    ws = T.workspace_for(ds, cam, K, entry_capacity=cap)
    out = T.build_mpi(ctx(), ds, cam, K, binning, rng, dtype=dtype, workspace=ws)
    info, st = T.build_stats(ctx(), ws, check=False)
    return out, info, st


def _check_partition(out, part, n):
    torch.cuda.synchronize()
    co = out["chunk_of"].cpu().numpy()[:n]
    assert np.array_equal(co, part.chunk_of)
    assert np.array_equal(out["chunk_count"].cpu().numpy(), part.chunk_count)
    assert np.array_equal(out["depth"].cpu().numpy().view(np.uint32), part.depth.view(np.uint32))


def _rotated_camera():
    from oracle.project import quat_to_rot
    R = quat_to_rot(np.array([[0.97, 0.1, -0.2, 0.05]]))[0]
    return scenegen.camera(160, 120, 50.0, 3.0, math.radians(25.0), R=R, t=(0.1, -0.05, 0.2))


PART_CASES = [
    ("uniform10k_invdepth", lambda: (scenegen.uniform_scene(10_000, 0), scenegen.config_camera("uniform10k")[0], 16,
                                     "inv_depth", (2.0, 6.0))),
    ("cluster50k_q64", lambda: (scenegen.cluster_scene(50_000, seed=3), scenegen.camera(256, 256, 50.0, 2.0, math.radians(40)),
                                64, "quantile", None)),
    ("fewer_than_chunks", lambda: (scenegen.small_scene(5, 1), scenegen.camera(64, 64, 50.0, 2.0, math.radians(20)), 16,
                                   "quantile", None)),
    ("rotated_camera", lambda: (scenegen.small_scene(3000, 2, xy=2.0, z=(-1.0, 6.0)), _rotated_camera(), 24, "quantile",
                                None)),
]


@pytest.mark.parametrize("case", PART_CASES, ids=[c[0] for c in PART_CASES])
def test_partition_bit_exact(case):
    name, make = case
    scene, cam, K, binning, rng = make()
    if name == "rotated_camera":
        m = scene["means"]
        m[10:20, 2] = m[20:30, 2]            # duplicate keys (ties by index)
        m[30] = [np.nan, 0.0, 3.0]
        m[31] = [0.0, 0.0, np.inf]
    announce("partition", name)
    out, info, st = _gpu_build(scene, cam, K, binning, rng)
    assert st == L.LF_OK
    g = geometry.derive(cam)
    part = partition.partition(scene["means"], cam, g, K, binning, rng)
    assert info.n_visible == part.order.size
    _check_partition(out, part, scene["means"].shape[0])


def _masked_compare(got, ref, amb, tol, jump):
    err = np.abs(got - ref).max(axis=-1)
    bad = (err > tol) & ~amb
    assert not bad.any(), f"{bad.sum()} unmasked texels above {tol}: max {err[~amb].max()}"
    if amb.any():
        assert err[amb].max() <= jump, err[amb].max()
    return float(err[~amb].max()), float(amb.mean())


@pytest.mark.parametrize("pdt", ["f32", "f16", "bf16"])
def test_planes_uniform10k(pdt):
    """All 16 planes of the 10k-Gaussian inverse-depth workload at 128^2."""
    announce("planes uniform10k", pdt)
    scene, cam, cfg = scenegen.config("uniform10k")
    out, info, st = _gpu_build(scene, cam, 16, "inv_depth", (2.0, 6.0), dtype=TDT[pdt])
    assert st == L.LF_OK
    mpi = render.build_mpi_gaussians(scene, cam, 16, "inv_depth", (2.0, 6.0))
    _check_partition(out, mpi.part, 10_000)
    got = host(out["rgba"])
    if pdt == "f32":
        e, frac = _masked_compare(got, mpi.planes, mpi.ambiguous, 1e-4, 0.02)
        print("unmasked max-abs", e, "ambiguous texel fraction", frac)
    else:
        e, frac = _masked_compare(got, mpi.planes, mpi.ambiguous, 2e-3, 0.02)
        q = psnr(got[..., :3], mpi.planes[..., :3])
        print(pdt, "unmasked max-abs", e, "PSNR", q)
        assert q >= 50.0


def test_planes_uniform10k_u8():
    """UNORM8 planes (Sec. 5.1) of the 10k-Gaussian workload: every code equals the code of
    the oracle's FP64 texel, except within 0.05 code units of a rounding tie (one code
    either way) and at texels the 1/255 inclusion test makes ambiguous (within the jump of
    one threshold Gaussian)."""
    announce("planes uniform10k", "u8")
    scene, cam, cfg = scenegen.config("uniform10k")
    out, info, st = _gpu_build(scene, cam, 16, "inv_depth", (2.0, 6.0), dtype=torch.uint8)
    assert st == L.LF_OK
    mpi = render.build_mpi_gaussians(scene, cam, 16, "inv_depth", (2.0, 6.0))
    _check_partition(out, mpi.part, 10_000)
    got = out["rgba"].cpu().numpy().astype(np.int32)
    ref = quantize.unorm8(mpi.planes).astype(np.int32)
    d = np.abs(got - ref)
    amb = np.broadcast_to(mpi.ambiguous[..., None], d.shape)
    tie = quantize.near_tie(mpi.planes, 0.05)
    assert d[~amb & ~tie].max(initial=0) == 0
    assert d[~amb].max(initial=0) <= 1
    assert d[amb].max(initial=0) <= 6                       # 0.02 * 255
    print("u8 codes off by one near ties:", int((d[~amb] == 1).sum()), "of", int((~amb).sum()))


@pytest.mark.parametrize("interp", ["nearest", "bilinear"])
def test_frame_uniform10k(interp):
    """Build + composite of the 9-view light field (plain method, FP32)."""
    announce("frame uniform10k", interp)
    scene, cam, cfg = scenegen.config("uniform10k")
    out, info, st = _gpu_build(scene, cam, 16, "inv_depth", (2.0, 6.0))
    dx, dy, _, _ = geometry.quilt_views(cam, 9, 1)
    dx, dy = dx.astype(np.float32), dy.astype(np.float32)
    views = T.composite(ctx(), out["rgba"], out["depth"], cam, T.views_of(dx, dy), interp)
    mpi = render.build_mpi_gaussians(scene, cam, 16, "inv_depth", (2.0, 6.0))
    ref, amb = composite.composite(mpi.planes, mpi.depth, cam, mpi.geom, dx, dy, interp, mpi.ambiguous)
    e, frac = _masked_compare(host(views), ref, amb, 1e-4, 0.03)
    print("frame unmasked max-abs", e, "ambiguous pixel fraction", frac)
    assert frac < 0.01


def test_zero_baseline_identity_on_gpu():
    """phi = 0: every composited view equals the oracle's conventional render (any N_chunk)."""
    announce("zero baseline")
    cam = scenegen.camera(96, 96, 50.0, 2.0, 0.0)
    scene = scenegen.small_scene(400, 9)
    for K in (1, 4):
        out, info, st = _gpu_build(scene, cam, K)
        v = T.composite(ctx(), out["rgba"], out["depth"], cam, T.views_of([0.0, 0.0]), "nearest")
        mpi = render.build_mpi_gaussians(scene, cam, K)
        ref, amb = render.render_view(scene, cam, 0.0, 0.0, visible=mpi.part.visible)
        ref = np.concatenate([ref[..., :3], 1.0 - ref[..., 3:]], axis=-1)
        got = host(v)
        for j in range(2):
            _masked_compare(got[j], ref, amb, 1e-4, 0.03)


def test_capacity_overflow_is_reported():
    announce("capacity overflow")
    scene = scenegen.small_scene(2000, 4)
    cam = scenegen.camera(256, 256, 50.0, 2.0, math.radians(30))
    out, info, st = _gpu_build(scene, cam, 8, cap=1000)
    assert st == L.LF_ERR_CAPACITY and info.overflow == 1 and info.entries_needed > 1000
    need = info.entries_needed
    out, info, st = _gpu_build(scene, cam, 8, cap=need)
    assert st == L.LF_OK and info.entries_needed == need


def test_build_deterministic():
    scene = scenegen.cluster_scene(100_000, seed=8)
    cam = scenegen.camera(384, 384, 50.0, 2.0, math.radians(40))
    a, _, _ = _gpu_build(scene, cam, 32)
    b, _, _ = _gpu_build(scene, cam, 32)
    torch.cuda.synchronize()
    assert torch.equal(a["rgba"], b["rgba"]) and torch.equal(a["depth"], b["depth"])


@pytest.mark.parametrize("key_bits,tile_bits", [(4, 4), (11, 11), (7, 9)])
def test_sort_digit_widths_agree(key_bits, tile_bits, monkeypatch):
    """The depth sort and the tile sort are stable sorts of unique (key, index) orders, so any
    digit width gives the same planes, bit for bit, as the default (8 / 10 bits).  4 bits: 8
    depth passes of 16 digits and 3 tile passes (an odd count: result in the alternate
    arrays); 11 bits: 3 depth passes of 2048 digits (several digits per thread) and 1 tile
    pass of 1024 digits; 7 / 9 bits: a narrower last depth pass."""
    announce("sort digit widths", key_bits, tile_bits)
    scene = scenegen.cluster_scene(100_000, seed=8)
    cam = scenegen.camera(384, 384, 50.0, 2.0, math.radians(40))
    ref, info0, st0 = _gpu_build(scene, cam, 32)
    assert st0 == L.LF_OK
    monkeypatch.setenv("LF_KEY_DIGIT_BITS", str(key_bits))
    monkeypatch.setenv("LF_TILE_DIGIT_BITS", str(tile_bits))
    got, info, st = _gpu_build(scene, cam, 32)
    assert st == L.LF_OK, L.lf_last_error()
    assert info.entries_needed == info0.entries_needed and info.stalled == 0
    torch.cuda.synchronize()
    assert torch.equal(ref["chunk_of"], got["chunk_of"]) and torch.equal(ref["depth"], got["depth"])
    assert torch.equal(ref["rgba"], got["rgba"])


@pytest.mark.parametrize("shift", [0, 5, 12, 24])
def test_splat_item_blocks_agree(shift, monkeypatch):
    """The splat's work items (chunk-major) are dealt to the XCDs in 2^shift blocks of
    consecutive items (LF_SPLAT_ITEM_SHIFT; the default is 8).  Which work-group takes which
    item changes no item's arithmetic, so every block count gives the default's planes bit
    for bit: 0 is one contiguous run per XCD, 24 one item per block."""
    announce("splat item blocks", shift)
    scene = scenegen.cluster_scene(100_000, seed=8)
    cam = scenegen.camera(384, 384, 50.0, 2.0, math.radians(40))
    ref, info0, st0 = _gpu_build(scene, cam, 32)
    assert st0 == L.LF_OK
    monkeypatch.setenv("LF_SPLAT_ITEM_SHIFT", str(shift))
    got, info, st = _gpu_build(scene, cam, 32)
    assert st == L.LF_OK, L.lf_last_error()
    torch.cuda.synchronize()
    assert torch.equal(ref["rgba"], got["rgba"]) and torch.equal(ref["depth"], got["depth"])


def test_constant_filter_planes():
    """The camera's constant dilation (adaptive-filter ablation) reaches the splat: planes at
    P_s = 2 against the oracle's with the same constant, and a constant equal to the Eq. 8
    value gives the adaptive planes bit for bit."""
    announce("planes constant filter")
    scene = scenegen.small_scene(2000, 12)
    cam = scenegen.camera(64, 48, 50.0, 3.0, math.radians(20), plane_scale=2.0, dilation=0.3)
    out, info, st = _gpu_build(scene, cam, 4)
    assert st == L.LF_OK
    mpi = render.build_mpi_gaussians(scene, cam, 4)
    _masked_compare(host(out["rgba"]), mpi.planes, mpi.ambiguous, 1e-4, 0.02)
    adaptive = cam.with_(dilation=0.0)
    same = cam.with_(dilation=float(np.float32(geometry.derive(adaptive).f_dilation)))
    a, _, _ = _gpu_build(scene, adaptive, 4)
    b, _, _ = _gpu_build(scene, same, 4)
    torch.cuda.synchronize()
    if np.float32(geometry.derive(adaptive).f_dilation) == np.float32(geometry.derive(same).f_dilation):
        assert torch.equal(a["rgba"], b["rgba"])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16, torch.uint8])
def test_empty_field_fill_stays_in_planes(dtype):
    """An empty field clears exactly its planes: a guard region behind them is untouched."""
    scene = T.to_device({k: v[:0] for k, v in scenegen.small_scene(4, 0).items()})
    cam = scenegen.camera(32, 32, 50.0, 2.0, math.radians(20))
    info = L.lf_geometry(L.make_camera(cam))
    K, n = 3, 3 * info.plane_height * info.plane_width * 4
    buf = torch.full((n + 4096,), 7, dtype=dtype, device="cuda")
    out = dict(rgba=buf[:n].view(K, info.plane_height, info.plane_width, 4),
               depth=torch.empty(K, dtype=torch.float32, device="cuda"))
    T.build_mpi(ctx(), scene, cam, K, dtype=dtype, out=out)
    torch.cuda.synchronize()
    assert float(buf[:n].float().abs().max()) == 0.0
    assert bool((buf[n:] == 7).all())


def test_empty_field():
    scene = {k: v[:0] for k, v in scenegen.small_scene(4, 0).items()}
    cam = scenegen.camera(32, 32, 50.0, 2.0, math.radians(20))
    out, info, st = _gpu_build(scene, cam, 4)
    assert st == L.LF_OK and info.n_visible == 0
    torch.cuda.synchronize()
    assert float(out["rgba"].abs().max()) == 0.0
    assert np.all(out["depth"].cpu().numpy() == np.float32(cam.d_focal))


BIN_CASES = [
    ("uniform10k_invdepth", lambda: (scenegen.uniform_scene(10_000, 0), scenegen.config_camera("uniform10k")[0], 16,
                                     "inv_depth", (2.0, 6.0))),
    ("cluster50k_q64_ragged", lambda: (scenegen.cluster_scene(50_000, seed=3),
                                       scenegen.camera(250, 200, 50.0, 2.0, math.radians(40)), 64, "quantile", None)),
    ("rotated_camera", lambda: (scenegen.small_scene(3000, 2, xy=2.0, z=(-1.0, 6.0)), _rotated_camera(), 24, "quantile",
                                None)),
]


@pytest.mark.parametrize("case", BIN_CASES, ids=[c[0] for c in BIN_CASES])
def test_tile_lists_against_oracle(case):
    """The (tile, chunk) lists (Sec. 4.4, Alg. 1 "Rasterize"): every list holds each Gaussian
    of its chunk whose support box meets the tile, in (key, index) order, and nothing beyond
    that box widened by 3e-3 relative and 3e-3 texel (the kernel's float32 margin)."""
    from oracle import bins
    name, make = case
    scene, cam, K, binning, rng = make()
    announce("tile lists", name)
    ds = T.to_device(scene)
    ws = T.workspace_for(ds, cam, K)
    T.build_mpi(ctx(), ds, cam, K, binning, rng, workspace=ws)
    tile, tx, ty, starts, entries = T.tile_lists(ctx(), ds, cam, K, ws)
    g = geometry.derive(cam)
    part = partition.partition(scene["means"], cam, g, K, binning, rng)
    must, may = bins.tile_lists(scene, cam, g, part, tile=tile)
    torch.cuda.synchronize()
    stats = bins.check_lists(starts.cpu().numpy(), entries.cpu().numpy(), must, may, part, tx * ty * K, K)
    print(name, stats)


@pytest.mark.parametrize("case", BIN_CASES, ids=[c[0] for c in BIN_CASES])
def test_splat_work_counts(case):
    """lf_build_splat_work: the support pairs equal the oracle's count of (Gaussian, texel)
    pairs with o G >= 1/255 (Sec. 4.4) up to the pairs within rounding of the threshold; the
    splat's evaluations cover every support pair and lie within the list texels, which are
    the entries x 256."""
    name, make = case
    scene, cam, K, binning, rng = make()
    announce("splat work counts", name)
    ds = T.to_device(scene)
    ws = T.workspace_for(ds, cam, K)
    T.build_mpi(ctx(), ds, cam, K, binning, rng, workspace=ws)
    w = T.splat_work(ctx(), ds, cam, K, ws)
    info, _ = T.build_stats(ctx(), ws, check=True)
    g = geometry.derive(cam)
    part = partition.partition(scene["means"], cam, g, K, binning, rng)
    want, near = 0, 0
    for k in range(K):
        got_k = splat.support_pairs(render.chunk_projection(scene, cam, g, part, k), g.hp, g.wp)
        want += got_k[0]
        near += got_k[1]
    print(name, w, "oracle support pairs", want, "near the threshold", near, flush=True)
    assert abs(w["support_pairs"] - want) <= near
    assert w["list_texels"] == int(info.entries_needed) * 256
    assert w["support_pairs"] <= w["evaluations"] <= w["list_texels"]
