"""ctypes binding of ``include/lf.h`` (argument marshalling only).

Every function here has the name of the C entry point it calls and raises
:class:`LFError` when the call returns a status other than ``LF_OK``.  Device
pointers are plain integers (e.g. ``tensor.data_ptr()``); streams are integers
(``torch.cuda.current_stream().cuda_stream``) or 0 for the null stream.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LF_LIBRARY") or os.path.join(HERE, "liblf.so")   # LF_LIBRARY: another build

LF_OK, LF_ERR_INVALID_ARG, LF_ERR_UNSUPPORTED, LF_ERR_CAPACITY, LF_ERR_OUT_OF_MEMORY, LF_ERR_HIP = range(6)
LF_F32, LF_F16, LF_BF16, LF_U8 = 0, 1, 2, 3
LF_NEAREST, LF_BILINEAR = 0, 1
LF_BIN_QUANTILE, LF_BIN_INV_DEPTH = 0, 1
LF_GAUSSIANS, LF_VOXELS = 0, 1
LF_MAX_VIEWS, LF_MAX_CHUNKS, LF_MAX_RES = 256, 4096, 8192

STATUS_NAMES = {0: "LF_OK", 1: "LF_ERR_INVALID_ARG", 2: "LF_ERR_UNSUPPORTED", 3: "LF_ERR_CAPACITY",
                4: "LF_ERR_OUT_OF_MEMORY", 5: "LF_ERR_HIP"}

# every symbol include/lf.h declares
EXPORTS = [
    "lf_version", "lf_last_error", "lf_create", "lf_destroy", "lf_geometry", "lf_quilt_views",
    "lf_build_mpi_workspace", "lf_build_mpi", "lf_build_stats", "lf_composite", "lf_composite_backward",
    "lf_build_mpi_backward", "lf_plane_coeffs", "lf_batch_create", "lf_batch_run", "lf_batch_stats", "lf_batch_group",
    "lf_batch_tile",
    "lf_batch_destroy", "lf_profile_enable", "lf_profile_read", "lf_render_view_workspace", "lf_render_view",
    "lf_sh_texel_floats", "lf_build_mpi_sh", "lf_composite_sh", "lf_sh_colours", "lf_build_tile_lists",
    "lf_build_splat_work", "lf_composite_noalloc",
]
LF_COMPOSITE_SCRATCH_BYTES = 4 << 20
LF_MAX_SH_DEGREE = 3
LF_BATCH_GRAPH, LF_BATCH_AUTOTUNE, LF_BATCH_WORKLIST = 1, 2, 4
PHASES = ["preprocess", "sort", "bin", "splat", "merge", "filter", "coeff", "composite", "composite_bwd",
          "build_bwd"]


class LFError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class lf_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("nx", C.c_int32), ("ny", C.c_int32),
                ("fov_x", C.c_float), ("fov_y", C.c_float), ("d_focal", C.c_float), ("phi_x", C.c_float),
                ("phi_y", C.c_float), ("d_shift", C.c_float), ("plane_scale", C.c_float), ("z_near", C.c_float),
                ("dilation", C.c_float)]


class lf_view(C.Structure):
    _fields_ = [("dx", C.c_float), ("dy", C.c_float)]


class lf_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("rgb", C.c_void_p), ("ijk", C.c_void_p), ("density", C.c_void_p),
                ("origin", C.c_float * 3), ("voxel_size", C.c_float)]


class lf_mpi(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("n_chunk", C.c_int32), ("height", C.c_int32), ("width", C.c_int32),
                ("rgba", C.c_void_p), ("depth", C.c_void_p), ("chunk_of", C.c_void_p),
                ("chunk_count", C.c_void_p)]


class lf_sh_mpi(C.Structure):
    _fields_ = [("degree", C.c_int32), ("n_chunk", C.c_int32), ("height", C.c_int32), ("width", C.c_int32),
                ("planes", C.c_void_p), ("depth", C.c_void_p)]


class lf_geometry_info(C.Structure):
    _fields_ = [("d_forward0", C.c_double), ("d_forward", C.c_double),
                ("tan_half_theta_prime_x", C.c_double), ("tan_half_theta_prime_y", C.c_double),
                ("f_dilation", C.c_double), ("fpx", C.c_double), ("fpy", C.c_double), ("cpx", C.c_double),
                ("cpy", C.c_double), ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("plane_width", C.c_int32), ("plane_height", C.c_int32),
                ("d_forward32", C.c_float), ("guard_x32", C.c_float), ("guard_y32", C.c_float),
                ("ratio_x32", C.c_float), ("ratio_y32", C.c_float), ("fpx32", C.c_float), ("fpy32", C.c_float),
                ("cpx32", C.c_float), ("cpy32", C.c_float), ("cx32", C.c_float), ("cy32", C.c_float),
                ("inv_focal32", C.c_float)]


class lf_build_info(C.Structure):
    _fields_ = [("n_visible", C.c_int64), ("entries_needed", C.c_int64), ("entry_capacity", C.c_int64),
                ("overflow", C.c_int32), ("stalled", C.c_int32)]


class lf_batch_item(C.Structure):
    _fields_ = [("field", lf_field), ("cam", lf_camera), ("n_chunk", C.c_int32), ("binning", C.c_int32),
                ("inv_depth_range", C.c_float * 2), ("views", C.POINTER(lf_view)), ("n_views", C.c_int32),
                ("interp", C.c_int32), ("out_dtype", C.c_int32), ("mpi", lf_mpi), ("out", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t)]


class lf_gaussian_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p), ("opacity", C.c_void_p),
                ("rgb", C.c_void_p)]


_lib = None


def load():
    """Load ``liblf.so``; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2508_18540_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "lf_version": ([], C.c_char_p),
        "lf_last_error": ([], C.c_char_p),
        "lf_create": ([C.POINTER(P), C.c_int], C.c_int),
        "lf_destroy": ([P], None),
        "lf_geometry": ([C.POINTER(lf_camera), C.POINTER(lf_geometry_info)], C.c_int),
        "lf_quilt_views": ([C.POINTER(lf_camera), C.c_int32, C.c_int32, C.POINTER(lf_view)], C.c_int),
        "lf_build_mpi_workspace": ([C.POINTER(lf_field), C.POINTER(lf_camera), C.c_int32, C.c_int64,
                                    C.POINTER(C.c_size_t)], C.c_int),
        "lf_build_mpi": ([P, C.POINTER(lf_field), C.POINTER(lf_camera), C.c_int32, C.c_int32,
                          C.POINTER(C.c_float), C.POINTER(lf_mpi), P, C.c_size_t, P], C.c_int),
        "lf_build_stats": ([P, P, C.c_size_t, C.POINTER(lf_build_info), P], C.c_int),
        "lf_build_tile_lists": ([P, C.POINTER(lf_field), C.POINTER(lf_camera), C.c_int32, P, C.c_size_t,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32), P, P, P], C.c_int),
        "lf_build_splat_work": ([P, C.POINTER(lf_field), C.POINTER(lf_camera), C.c_int32, P, C.c_size_t, P, P],
                                C.c_int),
        "lf_composite": ([P, C.POINTER(lf_mpi), C.POINTER(lf_camera), C.POINTER(lf_view), C.c_int32, C.c_int32,
                          C.c_int32, P, P], C.c_int),
        "lf_composite_noalloc": ([P, C.POINTER(lf_mpi), C.POINTER(lf_camera), C.POINTER(lf_view), C.c_int32,
                                  C.c_int32, C.c_int32, P, P], C.c_int),
        "lf_composite_backward": ([P, C.POINTER(lf_mpi), C.POINTER(lf_camera), C.POINTER(lf_view), C.c_int32,
                                   C.c_int32, P, P, P], C.c_int),
        "lf_build_mpi_backward": ([P, C.POINTER(lf_field), C.POINTER(lf_camera), C.POINTER(lf_mpi), P,
                                   C.POINTER(lf_gaussian_grads), P, C.c_size_t, P], C.c_int),
        "lf_batch_create": ([P, C.POINTER(lf_batch_item), C.c_int32, C.c_int32, C.POINTER(P)], C.c_int),
        "lf_batch_run": ([P, P], C.c_int),
        "lf_batch_stats": ([P, C.POINTER(lf_build_info), C.POINTER(C.c_int32), P], C.c_int),
        "lf_batch_group": ([P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
        "lf_batch_tile": ([P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
        "lf_batch_destroy": ([P], None),
        "lf_plane_coeffs": ([P, C.POINTER(lf_mpi), C.POINTER(lf_camera), C.POINTER(lf_view), C.c_int32,
                             P, P, P, P, P, P, P], C.c_int),
        "lf_render_view_workspace": ([C.POINTER(lf_field), C.POINTER(lf_camera), C.POINTER(C.c_size_t)], C.c_int),
        "lf_render_view": ([P, C.POINTER(lf_field), C.POINTER(lf_camera), C.POINTER(lf_view), C.POINTER(lf_mpi), P,
                            C.c_size_t, P], C.c_int),
        "lf_profile_enable": ([P, C.c_int32], C.c_int),
        "lf_sh_texel_floats": ([C.c_int32], C.c_int32),
        "lf_build_mpi_sh": ([P, C.POINTER(lf_field), P, C.POINTER(lf_camera), C.c_int32, C.c_int32,
                             C.POINTER(C.c_float), C.POINTER(lf_sh_mpi), P, C.c_size_t, P], C.c_int),
        "lf_composite_sh": ([P, C.POINTER(lf_sh_mpi), C.POINTER(lf_camera), C.POINTER(lf_view), C.c_int32,
                             C.c_int32, P, P], C.c_int),
        "lf_sh_colours": ([P, P, P, C.c_int32, C.c_int64, C.POINTER(lf_camera), C.POINTER(lf_view), P, P], C.c_int),
        "lf_profile_read": ([P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32], C.c_int),
    }
    for name, (args, res) in sig.items():
        if not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != LF_OK:
        raise LFError(status, where, load().lf_last_error().decode())


# ------------------------------------------------------------------------------------------
# struct builders
# ------------------------------------------------------------------------------------------

def make_camera(cam) -> lf_camera:
    """An ``lf_camera`` from any object with the fields of ``scenegen.Camera``."""
    c = lf_camera()
    c.R[:] = [float(v) for v in cam.R]
    c.t[:] = [float(v) for v in cam.t]
    c.nx, c.ny = int(cam.nx), int(cam.ny)
    for f in ("fov_x", "fov_y", "d_focal", "phi_x", "phi_y", "d_shift", "plane_scale", "z_near"):
        setattr(c, f, float(getattr(cam, f)))
    c.dilation = float(getattr(cam, "dilation", 0.0))
    return c


def make_views(dx, dy):
    n = len(dx)
    arr = (lf_view * n)()
    for i in range(n):
        arr[i].dx = float(dx[i])
        arr[i].dy = float(dy[i])
    return arr


def make_mpi(dtype: int, n_chunk: int, height: int, width: int, rgba: int, depth: int,
             chunk_of: int = 0, chunk_count: int = 0) -> lf_mpi:
    m = lf_mpi()
    m.dtype, m.n_chunk, m.height, m.width = dtype, n_chunk, height, width
    m.rgba, m.depth = rgba or None, depth or None
    m.chunk_of, m.chunk_count = chunk_of or None, chunk_count or None
    return m


# ------------------------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ------------------------------------------------------------------------------------------

def lf_version() -> str:
    return load().lf_version().decode()


def lf_last_error() -> str:
    return load().lf_last_error().decode()


def lf_create(device: int = 0) -> int:
    h = C.c_void_p()
    _check(load().lf_create(C.byref(h), device), "lf_create")
    return h.value


def lf_destroy(ctx: int) -> None:
    load().lf_destroy(ctx)


def lf_geometry(cam: lf_camera) -> lf_geometry_info:
    out = lf_geometry_info()
    _check(load().lf_geometry(C.byref(cam), C.byref(out)), "lf_geometry")
    return out


def lf_quilt_views(cam: lf_camera, vx: int, vy: int):
    out = (lf_view * (vx * vy))()
    _check(load().lf_quilt_views(C.byref(cam), vx, vy, out), "lf_quilt_views")
    return out


def lf_build_mpi_workspace(field: lf_field, cam: lf_camera, n_chunk: int, entry_capacity: int = 0) -> int:
    n = C.c_size_t()
    _check(load().lf_build_mpi_workspace(C.byref(field), C.byref(cam), n_chunk, entry_capacity, C.byref(n)),
           "lf_build_mpi_workspace")
    return n.value


def lf_build_mpi(ctx: int, field: lf_field, cam: lf_camera, n_chunk: int, binning: int, inv_depth_range,
                 mpi: lf_mpi, workspace: int, workspace_bytes: int, stream: int = 0) -> None:
    rng = None
    if inv_depth_range is not None:
        rng = (C.c_float * 2)(*[float(v) for v in inv_depth_range])
    _check(load().lf_build_mpi(ctx, C.byref(field), C.byref(cam), n_chunk, binning, rng, C.byref(mpi),
                               workspace, workspace_bytes, stream), "lf_build_mpi")


def lf_sh_texel_floats(degree: int) -> int:
    return int(load().lf_sh_texel_floats(degree))


def lf_build_mpi_sh(ctx: int, field: lf_field, sh: int, cam: lf_camera, n_chunk: int, binning: int, inv_depth_range,
                    mpi: lf_sh_mpi, workspace: int, workspace_bytes: int, stream: int = 0) -> None:
    rng = None
    if inv_depth_range is not None:
        rng = (C.c_float * 2)(*[float(v) for v in inv_depth_range])
    _check(load().lf_build_mpi_sh(ctx, C.byref(field), sh, C.byref(cam), n_chunk, binning, rng, C.byref(mpi),
                                  workspace, workspace_bytes, stream), "lf_build_mpi_sh")


def lf_composite_sh(ctx: int, mpi: lf_sh_mpi, cam: lf_camera, views, interp: int, out: int, stream: int = 0) -> None:
    _check(load().lf_composite_sh(ctx, C.byref(mpi), C.byref(cam), views, len(views), interp, out, stream),
           "lf_composite_sh")


def lf_sh_colours(ctx: int, means: int, sh: int, degree: int, n: int, cam: lf_camera, dx: float, dy: float,
                  rgb_out: int, stream: int = 0) -> None:
    v = lf_view(float(dx), float(dy))
    _check(load().lf_sh_colours(ctx, means, sh, degree, n, C.byref(cam), C.byref(v), rgb_out, stream),
           "lf_sh_colours")


def lf_render_view_workspace(field: lf_field, cam: lf_camera) -> int:
    n = C.c_size_t()
    _check(load().lf_render_view_workspace(C.byref(field), C.byref(cam), C.byref(n)), "lf_render_view_workspace")
    return n.value


def lf_render_view(ctx: int, field: lf_field, cam: lf_camera, dx: float, dy: float, out: lf_mpi, workspace: int,
                   workspace_bytes: int, stream: int = 0) -> None:
    v = lf_view(float(dx), float(dy))
    _check(load().lf_render_view(ctx, C.byref(field), C.byref(cam), C.byref(v), C.byref(out), workspace,
                                 workspace_bytes, stream), "lf_render_view")


def lf_build_stats(ctx: int, workspace: int, workspace_bytes: int, stream: int = 0, check: bool = True):
    out = lf_build_info()
    st = load().lf_build_stats(ctx, workspace, workspace_bytes, C.byref(out), stream)
    if check:
        _check(st, "lf_build_stats")
    return out, st


def lf_build_tile_lists(ctx: int, field: lf_field, cam: lf_camera, n_chunk: int, workspace: int, workspace_bytes: int,
                        bucket_start: int = 0, entries: int = 0, stream: int = 0):
    """Returns (tile, tiles_x, tiles_y); fills the device arrays when given."""
    t, tx, ty = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().lf_build_tile_lists(ctx, C.byref(field), C.byref(cam), n_chunk, workspace, workspace_bytes,
                                      C.byref(t), C.byref(tx), C.byref(ty), bucket_start or None, entries or None,
                                      stream), "lf_build_tile_lists")
    return t.value, tx.value, ty.value


def lf_build_splat_work(ctx: int, field: lf_field, cam: lf_camera, n_chunk: int, workspace: int,
                        workspace_bytes: int, counts: int, stream: int = 0) -> None:
    """Fills the device int64[3] counts (support pairs, evaluations, list entries x 256)."""
    _check(load().lf_build_splat_work(ctx, C.byref(field), C.byref(cam), n_chunk, workspace, workspace_bytes,
                                      counts, stream), "lf_build_splat_work")


def lf_composite(ctx: int, mpi: lf_mpi, cam: lf_camera, views, interp: int, out_dtype: int, out: int,
                 stream: int = 0) -> None:
    _check(load().lf_composite(ctx, C.byref(mpi), C.byref(cam), views, len(views), interp, out_dtype, out, stream),
           "lf_composite")


def lf_composite_noalloc(ctx: int, mpi: lf_mpi, cam: lf_camera, views, interp: int, out_dtype: int, out: int,
                         stream: int = 0) -> None:
    _check(load().lf_composite_noalloc(ctx, C.byref(mpi), C.byref(cam), views, len(views), interp, out_dtype, out,
                                       stream), "lf_composite_noalloc")


def lf_composite_backward(ctx: int, mpi: lf_mpi, cam: lf_camera, views, interp: int, d_out: int, d_planes: int,
                          stream: int = 0) -> None:
    _check(load().lf_composite_backward(ctx, C.byref(mpi), C.byref(cam), views, len(views), interp, d_out, d_planes,
                                        stream), "lf_composite_backward")


def lf_build_mpi_backward(ctx: int, field: lf_field, cam: lf_camera, mpi: lf_mpi, d_planes: int,
                          grads: lf_gaussian_grads, workspace: int, workspace_bytes: int, stream: int = 0) -> None:
    _check(load().lf_build_mpi_backward(ctx, C.byref(field), C.byref(cam), C.byref(mpi), d_planes, C.byref(grads),
                                        workspace, workspace_bytes, stream), "lf_build_mpi_backward")


def lf_plane_coeffs(ctx: int, mpi: lf_mpi, cam: lf_camera, views, bx: int, by: int, cx: int, cy: int,
                    cxn: int, cyn: int, stream: int = 0) -> None:
    _check(load().lf_plane_coeffs(ctx, C.byref(mpi), C.byref(cam), views, len(views), bx, by, cx, cy, cxn, cyn,
                                  stream), "lf_plane_coeffs")


def lf_batch_create(ctx: int, items, flags: int = 0) -> int:
    arr = (lf_batch_item * len(items))(*items)
    h = C.c_void_p()
    _check(load().lf_batch_create(ctx, arr, len(items), flags, C.byref(h)), "lf_batch_create")
    return h.value


def lf_batch_run(batch: int, stream: int = 0) -> None:
    _check(load().lf_batch_run(batch, stream), "lf_batch_run")


def lf_batch_stats(batch: int, n_items: int, stream: int = 0, check: bool = True):
    """(list of lf_build_info per scene, number of failed scenes, status)."""
    out = (lf_build_info * n_items)()
    nf = C.c_int32()
    st = load().lf_batch_stats(batch, out, C.byref(nf), stream)
    if check:
        _check(st, "lf_batch_stats")
    return list(out), nf.value, st


def lf_batch_group(batch: int, item: int) -> int:
    g = C.c_int32()
    _check(load().lf_batch_group(batch, item, C.byref(g)), "lf_batch_group")
    return g.value


def lf_batch_tile(batch: int, item: int) -> int:
    t = C.c_int32()
    _check(load().lf_batch_tile(batch, item, C.byref(t)), "lf_batch_tile")
    return t.value


def lf_batch_destroy(batch: int) -> None:
    load().lf_batch_destroy(batch)


def lf_profile_enable(ctx: int, enable: bool) -> None:
    _check(load().lf_profile_enable(ctx, 1 if enable else 0), "lf_profile_enable")


def lf_profile_read(ctx: int, reset: bool = True) -> dict:
    """{phase: (total_ms, count)} since the last reset (synchronises the device)."""
    ms = (C.c_double * len(PHASES))()
    cnt = (C.c_int64 * len(PHASES))()
    _check(load().lf_profile_read(ctx, ms, cnt, 1 if reset else 0), "lf_profile_read")
    return {p: (ms[i], cnt[i]) for i, p in enumerate(PHASES)}
