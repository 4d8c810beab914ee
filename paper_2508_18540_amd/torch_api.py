"""Torch-tensor front end of the C ABI: allocates outputs with torch, passes device pointers
and the current stream.  No compute happens here."""
from __future__ import annotations

import torch

from . import _lib as L

_DT = {torch.float32: L.LF_F32, torch.float16: L.LF_F16, torch.bfloat16: L.LF_BF16, torch.uint8: L.LF_U8}
_INTERP = {"nearest": L.LF_NEAREST, "bilinear": L.LF_BILINEAR}


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _need(t: torch.Tensor, name: str, dtypes=None, ndim=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtypes is not None and t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")


class Context:
    """An ``lf_ctx`` bound to one device."""

    def __init__(self, device: int | torch.device = 0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else device
        self.handle = L.lf_create(self.device.index or 0)

    def close(self):
        if self.handle:
            L.lf_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def views_of(dx, dy=None):
    if dy is None:
        dy = [0.0] * len(dx)
    return L.make_views(list(map(float, dx)), list(map(float, dy)))


def mpi_of(rgba: torch.Tensor, depth: torch.Tensor, chunk_of=None, chunk_count=None) -> L.lf_mpi:
    _need(rgba, "rgba", tuple(_DT), 4)
    _need(depth, "depth", (torch.float32,), 1)
    K, H, W, C = rgba.shape
    if C != 4 or depth.shape[0] != K:
        raise ValueError("rgba must be [K,H,W,4] and depth [K]")
    return L.make_mpi(_DT[rgba.dtype], K, H, W, rgba.data_ptr(), depth.data_ptr(),
                      chunk_of.data_ptr() if chunk_of is not None else 0,
                      chunk_count.data_ptr() if chunk_count is not None else 0)


def composite(ctx: Context, rgba: torch.Tensor, depth: torch.Tensor, cam, views, interp: str = "nearest",
              out_dtype=torch.float32, out: torch.Tensor | None = None) -> torch.Tensor:
    """lf_composite: returns views [V, ny, nx, 4] of (Q_r, Q_g, Q_b, T)."""
    m = mpi_of(rgba, depth)
    c = L.make_camera(cam)
    V = len(views)
    if out is None:
        out = torch.empty((V, cam.ny, cam.nx, 4), dtype=out_dtype, device=rgba.device)
    _need(out, "out", (torch.float32, torch.float16), 4)
    if tuple(out.shape) != (V, cam.ny, cam.nx, 4):
        raise ValueError(f"out must be [{V}, {cam.ny}, {cam.nx}, 4]")
    L.lf_composite(ctx.handle, m, c, views, _INTERP[interp], _DT[out.dtype], out.data_ptr(), _stream(rgba))
    return out


def plane_coeffs(ctx: Context, rgba: torch.Tensor, depth: torch.Tensor, cam, views):
    """lf_plane_coeffs: returns (bx, by, cx, cy, cxn, cyn) float32 tensors."""
    m = mpi_of(rgba, depth)
    K, V = depth.shape[0], len(views)
    dev = rgba.device
    bx, by = (torch.empty(K, dtype=torch.float32, device=dev) for _ in range(2))
    cs = [torch.empty((K, V), dtype=torch.float32, device=dev) for _ in range(4)]
    L.lf_plane_coeffs(ctx.handle, m, L.make_camera(cam), views, bx.data_ptr(), by.data_ptr(),
                      *[t.data_ptr() for t in cs], stream=_stream(rgba))
    return (bx, by, *cs)


_BIN = {"quantile": L.LF_BIN_QUANTILE, "inv_depth": L.LF_BIN_INV_DEPTH}
GAUSSIAN_KEYS = ("means", "log_scales", "quats", "opacity", "rgb")


def field_of(scene: dict) -> L.lf_field:
    """An lf_field over CUDA float32 tensors: Gaussians (means, log_scales, quats, opacity, rgb)."""
    f = L.lf_field()
    if "means" in scene:
        f.kind = L.LF_GAUSSIANS
        for k in GAUSSIAN_KEYS:
            _need(scene[k], k, (torch.float32,))
        f.n = scene["means"].shape[0]
        f.means, f.log_scales, f.quats, f.opacity, f.rgb = (scene[k].data_ptr() for k in GAUSSIAN_KEYS)
    else:
        f.kind = L.LF_VOXELS
        _need(scene["ijk"], "ijk", (torch.int32,))
        _need(scene["density"], "density", (torch.float32,))
        _need(scene["rgb"], "rgb", (torch.float32,))
        f.n = scene["ijk"].shape[0]
        f.ijk, f.density, f.rgb = scene["ijk"].data_ptr(), scene["density"].data_ptr(), scene["rgb"].data_ptr()
        f.origin[:] = [float(v) for v in scene["origin"]]
        f.voxel_size = float(scene["voxel_size"])
    return f


def to_device(scene: dict, device="cuda") -> dict:
    """Copy a scenegen scene (numpy) to CUDA tensors; scalars are kept as they are."""
    out = {}
    for k, v in scene.items():
        out[k] = torch.from_numpy(v).to(device) if hasattr(v, "dtype") and getattr(v, "ndim", 0) > 0 else v
    return out


class Workspace:
    """A device workspace for lf_build_mpi (a uint8 torch tensor)."""

    def __init__(self, nbytes: int, device):
        self.tensor = torch.empty(int(nbytes), dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return self.tensor.data_ptr()

    @property
    def nbytes(self):
        return self.tensor.numel()


def workspace_for(scene: dict, cam, n_chunk: int, entry_capacity: int = 0, device="cuda") -> Workspace:
    n = L.lf_build_mpi_workspace(field_of(scene), L.make_camera(cam), n_chunk, entry_capacity)
    return Workspace(n, device)


def build_mpi(ctx: Context, scene: dict, cam, n_chunk: int, binning: str = "quantile", inv_depth_range=None,
              dtype=torch.float32, workspace: Workspace | None = None, out: dict | None = None) -> dict:
    """lf_build_mpi: returns dict(rgba [K,H,W,4], depth [K], chunk_of [N], chunk_count [K], workspace)."""
    f = field_of(scene)
    c = L.make_camera(cam)
    info = L.lf_geometry(c)
    dev = ctx.device
    if workspace is None:
        workspace = workspace_for(scene, cam, n_chunk, device=dev)
    if out is None:
        out = dict(rgba=torch.empty((n_chunk, info.plane_height, info.plane_width, 4), dtype=dtype, device=dev),
                   depth=torch.empty(n_chunk, dtype=torch.float32, device=dev),
                   chunk_of=torch.empty(max(f.n, 1), dtype=torch.int32, device=dev),
                   chunk_count=torch.empty(n_chunk, dtype=torch.int32, device=dev))
    m = mpi_of(out["rgba"], out["depth"], out.get("chunk_of"), out.get("chunk_count"))
    L.lf_build_mpi(ctx.handle, f, c, n_chunk, _BIN[binning], inv_depth_range, m, workspace.ptr, workspace.nbytes,
                   torch.cuda.current_stream(dev).cuda_stream)
    out["workspace"] = workspace
    return out


def render_view(ctx: Context, scene: dict, cam, dx: float, dy: float = 0.0, dtype=torch.float32,
                workspace: Workspace | None = None, out: dict | None = None) -> dict:
    """lf_render_view: the conventional per-view render of view (dx, dy); returns dict(rgba
    [1, ny, nx, 4] premultiplied (C, 1 - T), depth [1], workspace)."""
    f = field_of(scene)
    c = L.make_camera(cam)
    dev = ctx.device
    if workspace is None:
        workspace = Workspace(L.lf_render_view_workspace(f, c), dev)
    if out is None:
        out = dict(rgba=torch.empty((1, cam.ny, cam.nx, 4), dtype=dtype, device=dev),
                   depth=torch.empty(1, dtype=torch.float32, device=dev))
    m = mpi_of(out["rgba"], out["depth"])
    L.lf_render_view(ctx.handle, f, c, dx, dy, m, workspace.ptr, workspace.nbytes,
                     torch.cuda.current_stream(dev).cuda_stream)
    out["workspace"] = workspace
    return out


def _sh_degree(sh: torch.Tensor) -> int:
    _need(sh, "sh", (torch.float32,), 3)
    nc = sh.shape[1]
    degree = int(round(nc ** 0.5)) - 1
    if (degree + 1) ** 2 != nc or sh.shape[2] != 3 or not 0 <= degree <= L.LF_MAX_SH_DEGREE:
        raise ValueError(f"sh must be [n, (L+1)^2, 3] with L <= {L.LF_MAX_SH_DEGREE}")
    return degree


def build_mpi_sh(ctx: Context, scene: dict, sh: torch.Tensor, cam, n_chunk: int, binning: str = "quantile",
                 inv_depth_range=None, workspace: Workspace | None = None, out: dict | None = None) -> dict:
    """lf_build_mpi_sh: SH planes of a Gaussian field; returns dict(planes [K,H,W,
    lf_sh_texel_floats(L)] float32, depth [K], degree, workspace)."""
    degree = _sh_degree(sh)
    if sh.shape[0] != scene["means"].shape[0]:
        raise ValueError("sh must have one row per Gaussian")
    f = field_of(scene)
    c = L.make_camera(cam)
    info = L.lf_geometry(c)
    dev = ctx.device
    if workspace is None:
        workspace = workspace_for(scene, cam, n_chunk, device=dev)
    tf = L.lf_sh_texel_floats(degree)
    if out is None:
        out = dict(planes=torch.empty((n_chunk, info.plane_height, info.plane_width, tf), dtype=torch.float32,
                                      device=dev),
                   depth=torch.empty(n_chunk, dtype=torch.float32, device=dev))
    _need(out["planes"], "planes", (torch.float32,), 4)
    if out["planes"].shape[3] != tf:
        raise ValueError(f"planes must have {tf} floats per texel for degree {degree}")
    m = L.lf_sh_mpi(degree, n_chunk, out["planes"].shape[1], out["planes"].shape[2], out["planes"].data_ptr(),
                    out["depth"].data_ptr())
    L.lf_build_mpi_sh(ctx.handle, f, sh.data_ptr(), c, n_chunk, _BIN[binning], inv_depth_range, m, workspace.ptr,
                      workspace.nbytes, torch.cuda.current_stream(dev).cuda_stream)
    out["degree"] = degree
    out["workspace"] = workspace
    return out


def composite_sh(ctx: Context, planes: torch.Tensor, depth: torch.Tensor, degree: int, cam, views,
                 interp: str = "nearest", out: torch.Tensor | None = None) -> torch.Tensor:
    """lf_composite_sh: views [V, ny, nx, 4] float32 of (Q_r, Q_g, Q_b, T) from SH planes."""
    _need(planes, "planes", (torch.float32,), 4)
    _need(depth, "depth", (torch.float32,), 1)
    if planes.shape[3] != L.lf_sh_texel_floats(degree) or depth.shape[0] != planes.shape[0]:
        raise ValueError("planes must be [K,H,W,lf_sh_texel_floats(degree)] and depth [K]")
    V = len(views)
    if out is None:
        out = torch.empty((V, cam.ny, cam.nx, 4), dtype=torch.float32, device=planes.device)
    _need(out, "out", (torch.float32,), 4)
    if tuple(out.shape) != (V, cam.ny, cam.nx, 4):
        raise ValueError(f"out must be [{V}, {cam.ny}, {cam.nx}, 4]")
    m = L.lf_sh_mpi(degree, planes.shape[0], planes.shape[1], planes.shape[2], planes.data_ptr(), depth.data_ptr())
    L.lf_composite_sh(ctx.handle, m, L.make_camera(cam), views, _INTERP[interp], out.data_ptr(), _stream(planes))
    return out


def sh_colours(ctx: Context, means: torch.Tensor, sh: torch.Tensor, cam, dx: float, dy: float = 0.0,
               out: torch.Tensor | None = None) -> torch.Tensor:
    """lf_sh_colours: every Gaussian's colour [n, 3] seen from view (dx, dy)."""
    degree = _sh_degree(sh)
    _need(means, "means", (torch.float32,), 2)
    if out is None:
        out = torch.empty((means.shape[0], 3), dtype=torch.float32, device=means.device)
    L.lf_sh_colours(ctx.handle, means.data_ptr(), sh.data_ptr(), degree, means.shape[0], L.make_camera(cam), dx, dy,
                    out.data_ptr(), _stream(means))
    return out


def render_view_sh(ctx: Context, scene: dict, sh: torch.Tensor, cam, dx: float, dy: float = 0.0,
                   workspace: Workspace | None = None, out: dict | None = None, rgb: torch.Tensor | None = None) -> dict:
    """The per-view render in SH colour: lf_sh_colours for the view, then lf_render_view."""
    rgb = sh_colours(ctx, scene["means"], sh, cam, dx, dy, out=rgb)
    return render_view(ctx, dict(scene, rgb=rgb), cam, dx, dy, workspace=workspace, out=out)


def build_stats(ctx: Context, workspace: Workspace, check: bool = True):
    """lf_build_stats (synchronises the current stream)."""
    info, status = L.lf_build_stats(ctx.handle, workspace.ptr, workspace.nbytes,
                                    torch.cuda.current_stream(ctx.device).cuda_stream, check=check)
    return info, status


def tile_lists(ctx: Context, scene: dict, cam, n_chunk: int, workspace: Workspace):
    """lf_build_tile_lists after a build_mpi on ``workspace``: (tile, tiles_x, tiles_y,
    bucket_start [tiles * n_chunk + 1] int64, entries [n] int32)."""
    f, c = field_of(scene), L.make_camera(cam)
    tile, tx, ty = L.lf_build_tile_lists(ctx.handle, f, c, n_chunk, workspace.ptr, workspace.nbytes)
    info, _ = build_stats(ctx, workspace)
    dev = ctx.device
    starts = torch.empty(tx * ty * n_chunk + 1, dtype=torch.int64, device=dev)
    entries = torch.empty(max(int(info.entries_needed), 1), dtype=torch.int32, device=dev)
    L.lf_build_tile_lists(ctx.handle, f, c, n_chunk, workspace.ptr, workspace.nbytes, starts.data_ptr(),
                          entries.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    return tile, tx, ty, starts, entries[:int(info.entries_needed)]


def splat_work(ctx: Context, scene: dict, cam, n_chunk: int, workspace: Workspace) -> dict:
    """lf_build_splat_work after a build_mpi on ``workspace``: the splat's support pairs,
    its (entry, texel) evaluations and the list entries x 256 texels."""
    counts = torch.empty(3, dtype=torch.int64, device=ctx.device)
    L.lf_build_splat_work(ctx.handle, field_of(scene), L.make_camera(cam), n_chunk, workspace.ptr, workspace.nbytes,
                          counts.data_ptr(), torch.cuda.current_stream(ctx.device).cuda_stream)
    c = counts.cpu().tolist()
    return {"support_pairs": c[0], "evaluations": c[1], "list_texels": c[2]}


def composite_backward(ctx: Context, rgba: torch.Tensor, depth: torch.Tensor, cam, views, d_out: torch.Tensor,
                       interp: str = "nearest", d_planes: torch.Tensor | None = None) -> torch.Tensor:
    """lf_composite_backward: dL/d(planes) [K, H, W, 4] float32 from dL/d(views) [V, ny, nx, 4]."""
    m = mpi_of(rgba, depth)
    _need(d_out, "d_out", (torch.float32,), 4)
    if tuple(d_out.shape) != (len(views), cam.ny, cam.nx, 4):
        raise ValueError(f"d_out must be [{len(views)}, {cam.ny}, {cam.nx}, 4]")
    if d_planes is None:
        d_planes = torch.empty(rgba.shape, dtype=torch.float32, device=rgba.device)
    _need(d_planes, "d_planes", (torch.float32,), 4)
    L.lf_composite_backward(ctx.handle, m, L.make_camera(cam), views, _INTERP[interp], d_out.data_ptr(),
                            d_planes.data_ptr(), _stream(rgba))
    return d_planes


def build_mpi_backward(ctx: Context, scene: dict, cam, out: dict, d_planes: torch.Tensor) -> dict:
    """lf_build_mpi_backward: gradients (means, log_scales, quats, opacity, rgb) of a Gaussian
    field from dL/d(planes), using the workspace of the build that produced ``out``."""
    f = field_of(scene)
    _need(d_planes, "d_planes", (torch.float32,), 4)
    if tuple(d_planes.shape) != tuple(out["rgba"].shape):
        raise ValueError("d_planes must have the planes' shape")
    grads = {k: torch.empty_like(scene[k]) for k in GAUSSIAN_KEYS}
    g = L.lf_gaussian_grads(*[grads[k].data_ptr() for k in GAUSSIAN_KEYS])
    m = mpi_of(out["rgba"], out["depth"])
    ws = out["workspace"]
    L.lf_build_mpi_backward(ctx.handle, f, L.make_camera(cam), m, d_planes.data_ptr(), g, ws.ptr, ws.nbytes,
                            torch.cuda.current_stream(ctx.device).cuda_stream)
    return grads


class LFRender(torch.autograd.Function):
    """Light field of a Gaussian field: lf_build_mpi then lf_composite forward, and
    lf_composite_backward then lf_build_mpi_backward backward.  Returns views
    [V, ny, nx, 4] = (Q_r, Q_g, Q_b, T) in float32; gradients flow to the five Gaussian
    parameter tensors.  Planes are kept (not recomputed) for the backward, with the build's
    workspace."""

    @staticmethod
    def forward(fctx, means, log_scales, quats, opacity, rgb, ctx, cam, views, n_chunk, interp="nearest",
                plane_dtype=torch.float32, binning="quantile", inv_depth_range=None, workspace=None):
        scene = dict(means=means.detach().contiguous(), log_scales=log_scales.detach().contiguous(),
                     quats=quats.detach().contiguous(), opacity=opacity.detach().contiguous(),
                     rgb=rgb.detach().contiguous())
        out = build_mpi(ctx, scene, cam, n_chunk, binning, inv_depth_range, dtype=plane_dtype, workspace=workspace)
        img = composite(ctx, out["rgba"], out["depth"], cam, views, interp)
        fctx.lf = (ctx, cam, views, interp, scene, out)
        return img

    @staticmethod
    def backward(fctx, d_img):
        ctx, cam, views, interp, scene, out = fctx.lf
        d_planes = composite_backward(ctx, out["rgba"], out["depth"], cam, views, d_img.contiguous().float(), interp)
        g = build_mpi_backward(ctx, scene, cam, out, d_planes)
        return (g["means"], g["log_scales"], g["quats"], g["opacity"], g["rgb"]) + (None,) * 9


def render_light_field(ctx: Context, params: dict, cam, views, n_chunk: int, interp: str = "nearest",
                       plane_dtype=torch.float32, binning: str = "quantile", inv_depth_range=None, workspace=None):
    """Differentiable light-field render of a Gaussian field (see LFRender)."""
    return LFRender.apply(params["means"], params["log_scales"], params["quats"], params["opacity"], params["rgb"],
                          ctx, cam, views, n_chunk, interp, plane_dtype, binning, inv_depth_range, workspace)


class Batch:
    """lf_batch over torch tensors: ``scenes`` is a list of dicts with keys scene (device
    field dict), cam, n_chunk, views (lf_view array), and optionally binning,
    inv_depth_range, interp, plane_dtype, out_dtype.  Allocates every scene's planes, views
    and workspace; ``run()`` renders them all (``outs[i]`` = dict(rgba, depth, chunk_of,
    chunk_count, views, workspace)), ``stats()`` reports every scene's build.  A scene's
    tile-list capacity is sized by one probe build unless ``probe`` (or the scene's own
    "probe" key) is false.  ``worklist`` runs the batch phase by phase (one splat, merge
    and composite launch over the work items of every scene) instead of one stream per
    scene."""

    def __init__(self, ctx: Context, scenes: list, graph: bool = True, autotune: bool = False, probe: bool = True,
                 worklist: bool = False):
        self.ctx = ctx
        self.outs, self._keep, items = [], [], []
        for sc in scenes:
            cam, K, views = sc["cam"], sc["n_chunk"], sc["views"]
            info = L.lf_geometry(L.make_camera(cam))
            dev = ctx.device
            ws = workspace_for(sc["scene"], cam, K, device=dev)
            if sc.get("probe", probe):
                # one build sizes the tile-list capacity (re-allocated once if the default is short)
                tmp = build_mpi(ctx, sc["scene"], cam, K, sc.get("binning", "quantile"), sc.get("inv_depth_range"),
                                dtype=sc.get("plane_dtype", torch.float16), workspace=ws)
                st_info, st = build_stats(ctx, ws, check=False)
                del tmp
                if st == L.LF_ERR_CAPACITY:
                    ws = workspace_for(sc["scene"], cam, K, entry_capacity=int(st_info.entries_needed * 1.25) + 1024,
                                       device=dev)
            o = dict(rgba=torch.empty((K, info.plane_height, info.plane_width, 4), dtype=sc.get("plane_dtype", torch.float16),
                                      device=dev),
                     depth=torch.empty(K, dtype=torch.float32, device=dev),
                     chunk_of=torch.empty(max(int(field_of(sc["scene"]).n), 1), dtype=torch.int32, device=dev),
                     chunk_count=torch.empty(K, dtype=torch.int32, device=dev),
                     views=torch.empty((len(views), cam.ny, cam.nx, 4), dtype=sc.get("out_dtype", torch.float32), device=dev),
                     workspace=ws)
            it = L.lf_batch_item()
            it.field = field_of(sc["scene"])
            it.cam = L.make_camera(cam)
            it.n_chunk = K
            it.binning = _BIN[sc.get("binning", "quantile")]
            if sc.get("inv_depth_range") is not None:
                it.inv_depth_range[:] = [float(v) for v in sc["inv_depth_range"]]
            it.views = views
            it.n_views = len(views)
            it.interp = _INTERP[sc.get("interp", "nearest")]
            it.out_dtype = _DT[o["views"].dtype]
            it.mpi = mpi_of(o["rgba"], o["depth"], o["chunk_of"], o["chunk_count"])
            it.out = o["views"].data_ptr()
            it.workspace = ws.ptr
            it.workspace_bytes = ws.nbytes
            items.append(it)
            self.outs.append(o)
            self._keep.append((sc, views))
        flags = ((L.LF_BATCH_GRAPH if graph else 0) | (L.LF_BATCH_AUTOTUNE if autotune else 0)
                 | (L.LF_BATCH_WORKLIST if worklist else 0))
        self.handle = L.lf_batch_create(ctx.handle, items, flags)

    def run(self):
        L.lf_batch_run(self.handle, torch.cuda.current_stream(self.ctx.device).cuda_stream)
        return self.outs

    def stats(self, check: bool = True):
        """lf_batch_stats after the last run: (per-scene lf_build_info list, failed scenes,
        status); raises on a failed scene when ``check``."""
        return L.lf_batch_stats(self.handle, len(self.outs), torch.cuda.current_stream(self.ctx.device).cuda_stream,
                                check)

    def groups(self):
        return [L.lf_batch_group(self.handle, i) for i in range(len(self.outs))]

    def tiles(self):
        return [L.lf_batch_tile(self.handle, i) for i in range(len(self.outs))]

    def close(self):
        if getattr(self, "handle", 0):
            L.lf_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
