// MPI build entry points (Alg. 1 steps 1-5): validation, workspace layout, launches.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "build_internal.h"
#include "sort_internal.h"

namespace lf {

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int splat_item_shift() {
  if (const char* e = getenv("LF_SPLAT_ITEM_SHIFT")) {
    const int v = atoi(e);
    if (v >= 0 && v <= 24) return v;
  }
  // 256 blocks: with the items chunk-major, a block is about a quarter of one plane.
  // Measured on the 500k-Gaussian frame (splat work-group reads, FETCH_SIZE, and splat
  // time): 256 blocks read 105 MB at 0.285-0.30 ms; 1024 blocks 138 MB at 0.276-0.29 ms; one item
  // per block (item i on XCD i mod 8) 203 MB at 0.32 ms; 128 blocks 98 MB at 0.31 ms.
  // (The splat backward deals the same items in blocks of its own.)
  return 8;
}

BuildLayout build_layout(int32_t kind, int64_t n, int32_t K, int32_t wp, int32_t hp, int64_t cap) {
  BuildLayout L;
  std::memset(&L, 0, sizeof(L));
  L.kind = kind;
  L.rec_bytes = kind == LF_VOXELS ? (int32_t)sizeof(VRec) : (int32_t)sizeof(GRec);
  if (kind == LF_VOXELS) {
    L.filt_bands = (hp + kFiltRows - 1) / kFiltRows;
    L.filt_segs = (wp + kFiltCols - 1) / kFiltCols;
  }
  L.n = n;
  L.cap = cap;
  L.K = K;
  L.ntx = (wp + kTile - 1) / kTile;
  L.nty = (hp + kTile - 1) / kTile;
  L.n_tiles = L.ntx * L.nty;
  L.n_buckets = (int64_t)L.n_tiles * K;
  int bits = 1;
  while ((1LL << bits) < L.n_tiles) ++bits;
  L.tile_bits = bits;
  bits = 0;
  while ((1LL << bits) < K) ++bits;
  L.chunk_bits = bits;                 // entry sort keys are (tile << chunk_bits) | chunk
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t un = (size_t)(n > 0 ? n : 1);
  L.o_hdr = take(sizeof(BuildHeader));
  L.o_sync = take((size_t)2 * kRadixHistWordsMax * 4 +
                  (scan_state_words((int64_t)un) + scan_state_words(L.n_buckets)) * 8);
  L.o_keys = take(un * 4);
  L.o_vals = take(un * 4);
  L.o_keys_alt = take(un * 4);
  L.o_vals_alt = take(un * 4);
  L.o_rec = take(un * (size_t)L.rec_bytes);
  L.o_ntiles_i = take(un * 4);
  L.o_ntiles_r = take(un * 8);
  L.o_chunk_r = take(un * 4);
  L.o_offsets = take((un + 1) * 8);
  L.o_chunk_start = take((size_t)(K + 1) * 8);
  L.o_edges = take((size_t)K * 4);
  L.o_dtab = take((size_t)K * 4);
  L.o_nseg = take((size_t)(L.n_buckets + 1) * 4);
  L.o_bucket = take((size_t)(L.n_buckets + 1) * 4);
  L.o_radix = take(radix_tmp_u32(n > cap ? n : cap) * 4);
  const size_t uc = (size_t)(cap > 0 ? cap : 1) + kEntryPad;
  L.o_ekeys = take(uc * 4);
  L.o_evals = take(uc * 4);
  L.o_ekeys_alt = take(uc * 4);
  L.o_evals_alt = take(uc * 4);
  L.o_heads = take(((size_t)(cap > 0 ? cap : 1) / 256 + 2) * 4);
  const int64_t segs = (cap + kSegment - 1) / kSegment;
  L.max_items = L.n_buckets + segs + 1;
  L.max_partial = 2 * segs + 16;
  L.o_pcnt = take((size_t)(L.n_buckets + 1) * 4);
  L.o_item_start = take((size_t)(L.n_buckets + 1) * 4);
  L.o_pslot = take((size_t)(L.n_buckets + 1) * 4);

  L.o_items = take((size_t)L.max_items * 8);
  L.o_partial = take((size_t)L.max_partial * kTile * kTile * 16);
  L.o_split = take((size_t)L.max_partial * 4);
  L.o_stage = take(kind == LF_VOXELS ? (size_t)K * hp * wp * 16 : 0);
  L.o_ggrad = take(kind == LF_VOXELS ? 0 : un * kGradSlots * 4);
  L.clear_words = (int64_t)(L.o_keys - L.o_hdr) / 4;   // header and sync region
  L.total = o;
  return L;
}

namespace {

constexpr int64_t kMaxPrimitives = (1LL << 28) - 1;   // entry values keep 28 index bits
constexpr int64_t kMaxEntries = (1LL << 31) - 1;
// per list entry: four u32 sort arrays, item records and 2/kSegment partial tiles of 4 KB
constexpr size_t kBytesPerEntry = 16 + 8 + 2 * kTile * kTile * 16 / kSegment + 1;

int64_t default_capacity(int64_t n) {
  const int64_t c = 16 * n;
  return c < 65536 ? 65536 : (c > kMaxEntries ? kMaxEntries : c);
}

// The largest entry capacity a workspace of `bytes` holds (0 if none).
int64_t capacity_of(int32_t kind, int64_t n, int32_t K, int32_t wp, int32_t hp, size_t bytes) {
  const size_t fixed = build_layout(kind, n, K, wp, hp, 0).total + radix_tmp_u32(kMaxEntries) * 4 + 4 * 256;
  if (bytes <= fixed) return 0;
  int64_t cap = (int64_t)((bytes - fixed) / kBytesPerEntry);
  if (cap > kMaxEntries) cap = kMaxEntries;
  while (cap > 0 && build_layout(kind, n, K, wp, hp, cap).total > bytes) cap -= 64;
  return cap > 0 ? cap : 0;
}

lf_status check_field(const lf_field* f) {
  if (!f) return fail(LF_ERR_INVALID_ARG, "field is NULL");
  if (f->n < 0 || f->n > kMaxPrimitives) return fail(LF_ERR_INVALID_ARG, "field size %lld outside [0, 2^28)", (long long)f->n);
  if (f->kind == LF_GAUSSIANS) {
    if (f->n > 0 && !(f->means && f->log_scales && f->quats && f->opacity && f->rgb))
      return fail(LF_ERR_INVALID_ARG, "a Gaussian attribute pointer is NULL");
    return LF_OK;
  }
  if (f->kind == LF_VOXELS) {
    if (f->n > 0 && !(f->ijk && f->density && f->rgb))
      return fail(LF_ERR_INVALID_ARG, "a voxel attribute pointer is NULL");
    if (!(std::isfinite(f->voxel_size) && f->voxel_size > 0.0f))
      return fail(LF_ERR_INVALID_ARG, "voxel_size must be finite and positive");
    if (!(std::isfinite(f->origin[0]) && std::isfinite(f->origin[1]) && std::isfinite(f->origin[2])))
      return fail(LF_ERR_INVALID_ARG, "voxel grid origin must be finite");
    return LF_OK;
  }
  return fail(LF_ERR_INVALID_ARG, "field kind %d is not GAUSSIANS/VOXELS", f->kind);
}

lf_status check_common(const lf_field* field, const lf_camera* cam, int32_t n_chunk, Geom* g) {
  lf_status s = check_field(field);
  if (s != LF_OK) return s;
  if ((s = derive_geometry(cam, g)) != LF_OK) return s;
  if (n_chunk < 1 || n_chunk > LF_MAX_CHUNKS)
    return fail(LF_ERR_INVALID_ARG, "n_chunk %d outside [1, %d]", n_chunk, LF_MAX_CHUNKS);
  return LF_OK;
}

// Kernel arguments of a build (or its backward) on `workspace` laid out as L.
void build_args(BuildArgs& a, const BuildLayout& L, const lf_field* field, const lf_camera* cam, const Geom& g,
                int32_t n_chunk, int32_t binning, const lf_mpi* mpi, void* workspace, int64_t cap) {
  const int64_t n = field->n;
  char* w = static_cast<char*>(workspace);
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.capacity = cap;
  a.K = n_chunk;
  a.ntx = L.ntx;
  a.n_tiles = L.n_tiles;
  a.chunk_bits = L.chunk_bits;
  a.kind = field->kind;
  a.rec_bytes = L.rec_bytes;
  a.filt_bands = L.filt_bands;
  a.filt_segs = L.filt_segs;
  a.binning = binning;
  a.plane_dtype = mpi->dtype;
  a.d_focal32 = cam->d_focal;
  a.c = g.c;
  a.means = field->means;
  a.log_scales = field->log_scales;
  a.quats = field->quats;
  a.opacity = field->opacity;
  a.rgb = field->rgb;
  a.planes = mpi->rgba;
  a.depth = mpi->depth;
  a.chunk_of = mpi->chunk_of;
  a.chunk_count = mpi->chunk_count;
  a.hdr = reinterpret_cast<BuildHeader*>(w + L.o_hdr);
  a.keys = reinterpret_cast<uint32_t*>(w + L.o_keys);
  a.vals = reinterpret_cast<uint32_t*>(w + L.o_vals);
  a.keys_alt = reinterpret_cast<uint32_t*>(w + L.o_keys_alt);
  a.vals_alt = reinterpret_cast<uint32_t*>(w + L.o_vals_alt);
  a.rec = reinterpret_cast<GRec*>(w + L.o_rec);
  a.ntiles_i = reinterpret_cast<uint32_t*>(w + L.o_ntiles_i);
  a.ntiles_r = reinterpret_cast<uint64_t*>(w + L.o_ntiles_r);
  a.chunk_r = reinterpret_cast<uint32_t*>(w + L.o_chunk_r);
  a.offsets = reinterpret_cast<uint64_t*>(w + L.o_offsets);
  a.chunk_start = reinterpret_cast<int64_t*>(w + L.o_chunk_start);
  a.edges = reinterpret_cast<float*>(w + L.o_edges);
  a.dtab = reinterpret_cast<float*>(w + L.o_dtab);
  a.nseg = reinterpret_cast<uint32_t*>(w + L.o_nseg);
  a.bucket = reinterpret_cast<uint32_t*>(w + L.o_bucket);
  a.radix_tmp = reinterpret_cast<uint32_t*>(w + L.o_radix);
  a.ghist_key = reinterpret_cast<uint32_t*>(w + L.o_sync);
  a.ghist_tile = a.ghist_key + kRadixHistWordsMax;
  a.scan_state_offsets = reinterpret_cast<uint64_t*>(a.ghist_tile + kRadixHistWordsMax);
  a.scan_state_items = a.scan_state_offsets + scan_state_words(L.n > 0 ? L.n : 1);
  a.clear_words = L.clear_words;
  a.ekeys = reinterpret_cast<uint32_t*>(w + L.o_ekeys);
  a.evals = reinterpret_cast<uint32_t*>(w + L.o_evals);
  a.ekeys_alt = reinterpret_cast<uint32_t*>(w + L.o_ekeys_alt);
  a.evals_alt = reinterpret_cast<uint32_t*>(w + L.o_evals_alt);
  a.heads = reinterpret_cast<uint32_t*>(w + L.o_heads);
  a.n_heads = (L.cap > 0 ? L.cap : 1) / 256 + 2;
  a.pcnt = reinterpret_cast<uint32_t*>(w + L.o_pcnt);
  a.item_start = reinterpret_cast<uint32_t*>(w + L.o_item_start);
  a.pslot = reinterpret_cast<uint32_t*>(w + L.o_pslot);
  a.split = reinterpret_cast<uint32_t*>(w + L.o_split);
  a.items = reinterpret_cast<uint2*>(w + L.o_items);
  a.partial = reinterpret_cast<float4*>(w + L.o_partial);
  a.max_items = L.max_items;
  a.item_shift = splat_item_shift();
  a.stage = reinterpret_cast<float4*>(w + L.o_stage);
  if (field->kind == LF_VOXELS) {
    a.ijk = field->ijk;
    a.density = field->density;
    a.rgb = field->rgb;
    for (int i = 0; i < 3; ++i) a.origin[i] = field->origin[i];
    a.vsize = field->voxel_size;
    a.inv_vsize = (float)(1.0 / (double)field->voxel_size);
    // reference camera centre in world cell units: (R^T ((0, 0, D_fwd) - t) - origin) / h
    const double h = field->voxel_size;
    const double oc[3] = {-(double)cam->t[0], -(double)cam->t[1], g.d_forward - (double)cam->t[2]};
    for (int i = 0; i < 3; ++i) {
      const double w_i = (double)cam->R[i] * oc[0] + (double)cam->R[3 + i] * oc[1] + (double)cam->R[6 + i] * oc[2];
      const double cell = (w_i - (double)field->origin[i]) / h;
      a.cam_cell[i] = (float)cell;
      a.cam_cell_lo[i] = (float)(cell - (double)a.cam_cell[i]);
    }
  }
  a.ggrad = reinterpret_cast<float*>(w + L.o_ggrad);
}

}  // namespace
}  // namespace lf

using namespace lf;

extern "C" lf_status lf_build_mpi_workspace(const lf_field* field, const lf_camera* cam, int32_t n_chunk,
                                            int64_t entry_capacity, size_t* bytes) {
  if (!bytes) return fail(LF_ERR_INVALID_ARG, "bytes is NULL");
  Geom g;
  lf_status s = check_common(field, cam, n_chunk, &g);
  if (s != LF_OK) return s;
  if (entry_capacity > kMaxEntries) return fail(LF_ERR_INVALID_ARG, "entry_capacity exceeds 2^31 - 1");
  const int64_t cap = entry_capacity > 0 ? entry_capacity : default_capacity(field->n);
  const size_t fixed =
      build_layout(field->kind, field->n, n_chunk, g.wp, g.hp, 0).total + radix_tmp_u32(kMaxEntries) * 4 + 4 * 256;
  *bytes = fixed + (size_t)cap * kBytesPerEntry + 4096;
  return LF_OK;
}

namespace lf {
namespace {

}  // namespace

lf_status build_prepare(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, int32_t n_chunk, int32_t binning,
                        const float* inv_depth_range, const lf_mpi* mpi, const float* sh, int32_t sh_coef,
                        void* workspace, size_t workspace_bytes, hipStream_t st, BuildArgs* out_a, BuildLayout* out_L) {
  Geom g;
  lf_status s = check_common(field, cam, n_chunk, &g);
  if (s != LF_OK) return s;
  if (binning != LF_BIN_QUANTILE && binning != LF_BIN_INV_DEPTH)
    return fail(LF_ERR_INVALID_ARG, "binning %d is not QUANTILE/INV_DEPTH", binning);
  float zlo = 0.f, zhi = 0.f;
  if (binning == LF_BIN_INV_DEPTH) {
    if (!inv_depth_range) return fail(LF_ERR_INVALID_ARG, "inv_depth_range is NULL");
    zlo = inv_depth_range[0];
    zhi = inv_depth_range[1];
    if (!(std::isfinite(zlo) && std::isfinite(zhi) && zlo < zhi && (double)zlo > g.d_forward))
      return fail(LF_ERR_INVALID_ARG, "inverse-depth range must satisfy D_forward < z_lo < z_hi < inf");
  }
  if (!mpi) return fail(LF_ERR_INVALID_ARG, "mpi is NULL");
  if (mpi->dtype != LF_F32 && mpi->dtype != LF_F16 && mpi->dtype != LF_BF16 && mpi->dtype != LF_U8)
    return fail(LF_ERR_INVALID_ARG, "mpi dtype %d is not F32/F16/BF16/U8", mpi->dtype);
  if (mpi->n_chunk != n_chunk) return fail(LF_ERR_INVALID_ARG, "mpi n_chunk %d != %d", mpi->n_chunk, n_chunk);
  if (mpi->width != g.wp || mpi->height != g.hp)
    return fail(LF_ERR_INVALID_ARG, "mpi is %dx%d but the camera's planes are %dx%d", mpi->width, mpi->height, g.wp,
                g.hp);
  if (!mpi->rgba || !mpi->depth) return fail(LF_ERR_INVALID_ARG, "mpi planes/depth is NULL");
  if (!workspace) return fail(LF_ERR_INVALID_ARG, "workspace is NULL");
  const int64_t n = field->n;
  const int64_t cap = capacity_of(field->kind, n, n_chunk, g.wp, g.hp, workspace_bytes);
  if (cap < 1) {
    size_t need = 0;
    lf_build_mpi_workspace(field, cam, n_chunk, 0, &need);
    return fail(LF_ERR_CAPACITY, "workspace of %zu bytes is too small; %zu bytes needed", workspace_bytes, need);
  }
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");

  const BuildLayout L = build_layout(field->kind, n, n_chunk, g.wp, g.hp, cap);
  if (L.tile_bits + L.chunk_bits > 32)
    return fail(LF_ERR_INVALID_ARG, "%d tiles x %d chunks do not fit a 32-bit (tile, chunk) key", L.n_tiles, n_chunk);
  BuildArgs a;
  build_args(a, L, field, cam, g, n_chunk, binning, mpi, workspace, cap);
  a.sh = sh;
  a.sh_coef = sh_coef;
  if (binning == LF_BIN_INV_DEPTH) {
    // K planes uniform in 1/z over [z_lo, z_hi]: interior edges E_i and plane depths at i = k + 1/2
    std::vector<float> edges((size_t)n_chunk, 0.0f), dtab((size_t)n_chunk);
    const double il = 1.0 / (double)zlo, ih = 1.0 / (double)zhi;
    for (int i = 1; i < n_chunk; ++i) edges[i - 1] = (float)(1.0 / (il + ((double)i / n_chunk) * (ih - il)));
    for (int k = 0; k < n_chunk; ++k) dtab[k] = (float)(1.0 / (il + (((double)k + 0.5) / n_chunk) * (ih - il)));
    if ((e = upload_table(a.edges, edges.data(), n_chunk, st)) != hipSuccess) return hip_fail(e, "table upload");
    if ((e = upload_table(a.dtab, dtab.data(), n_chunk, st)) != hipSuccess) return hip_fail(e, "table upload");
  }
  *out_a = a;
  *out_L = L;
  return LF_OK;
}

namespace {

// lf_build_mpi, and with sh / sh_coef > 0 the SH planes of lf_build_mpi_sh (mpi then
// describes float32 planes of sh_texel_floats(sh_coef) floats per texel).
lf_status build_mpi_impl(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, int32_t n_chunk, int32_t binning,
                         const float* inv_depth_range, lf_mpi* mpi, const float* sh, int32_t sh_coef, void* workspace,
                         size_t workspace_bytes, void* stream) {
  BuildArgs a;
  BuildLayout L;
  hipStream_t st = (hipStream_t)stream;
  lf_status s = build_prepare(ctx, field, cam, n_chunk, binning, inv_depth_range, mpi, sh, sh_coef, workspace,
                              workspace_bytes, st, &a, &L);
  if (s != LF_OK) return s;
  const hipError_t e = build_planes(a, L, st, &ctx->prof);
  if (e != hipSuccess) return hip_fail(e, "build launch");
  return LF_OK;
}

}  // namespace
}  // namespace lf

extern "C" lf_status lf_build_mpi(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, int32_t n_chunk,
                                  int32_t binning, const float* inv_depth_range, lf_mpi* mpi, void* workspace,
                                  size_t workspace_bytes, void* stream) {
  return build_mpi_impl(ctx, field, cam, n_chunk, binning, inv_depth_range, mpi, nullptr, 0, workspace,
                        workspace_bytes, stream);
}

extern "C" lf_status lf_build_mpi_sh(lf_ctx* ctx, const lf_field* field, const float* sh, const lf_camera* cam,
                                     int32_t n_chunk, int32_t binning, const float* inv_depth_range, lf_sh_mpi* mpi,
                                     void* workspace, size_t workspace_bytes, void* stream) {
  if (!field) return fail(LF_ERR_INVALID_ARG, "field is NULL");
  if (field->kind != LF_GAUSSIANS) return fail(LF_ERR_UNSUPPORTED, "SH planes cover Gaussian fields only");
  if (!mpi) return fail(LF_ERR_INVALID_ARG, "mpi is NULL");
  if (mpi->degree < 0 || mpi->degree > LF_MAX_SH_DEGREE)
    return fail(LF_ERR_INVALID_ARG, "SH degree %d outside [0, %d]", mpi->degree, LF_MAX_SH_DEGREE);
  if (field->n > 0 && !sh) return fail(LF_ERR_INVALID_ARG, "sh is NULL");
  // the RGB build over the SH planes: rgb is not read by the SH splat (preprocess copies
  // three floats per Gaussian into its records, which sh always holds)
  lf_field f = *field;
  if (!f.rgb) f.rgb = sh;
  lf_mpi m{LF_F32, mpi->n_chunk, mpi->height, mpi->width, mpi->planes, mpi->depth, nullptr, nullptr};
  return build_mpi_impl(ctx, &f, cam, n_chunk, binning, inv_depth_range, &m, sh, (mpi->degree + 1) * (mpi->degree + 1),
                        workspace, workspace_bytes, stream);
}

// The view camera of lf_render_view as a light-field camera with no baseline: D_forward = 0,
// theta' = theta, one plane at the view resolution, and the 0.3 texel^2 dilation of 3DGS.
static lf_camera view_camera(const lf_camera* cam) {
  lf_camera v = *cam;
  v.phi_x = v.phi_y = 0.0f;
  v.d_shift = 0.0f;
  v.plane_scale = 1.0f;
  v.dilation = 0.0f;     // Eq. 8 with no baseline and P_s = 1: the 0.3 px^2 of 3DGS
  return v;
}

extern "C" lf_status lf_render_view_workspace(const lf_field* field, const lf_camera* cam, size_t* bytes) {
  if (!cam) return fail(LF_ERR_INVALID_ARG, "camera is NULL");
  const lf_camera v = view_camera(cam);
  return lf_build_mpi_workspace(field, &v, 1, 0, bytes);
}

extern "C" lf_status lf_render_view(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, const lf_view* view,
                                    lf_mpi* out, void* workspace, size_t workspace_bytes, void* stream) {
  if (!cam) return fail(LF_ERR_INVALID_ARG, "camera is NULL");
  if (!view) return fail(LF_ERR_INVALID_ARG, "view is NULL");
  if (!(std::isfinite(view->dx) && std::isfinite(view->dy))) return fail(LF_ERR_INVALID_ARG, "view offset is not finite");
  const lf_camera vc = view_camera(cam);
  Geom g;
  lf_status s = check_common(field, &vc, 1, &g);
  if (s != LF_OK) return s;
  if (field->kind != LF_GAUSSIANS) return fail(LF_ERR_UNSUPPORTED, "the per-view render covers Gaussian fields only");
  if (!out) return fail(LF_ERR_INVALID_ARG, "out is NULL");
  if (out->dtype != LF_F32 && out->dtype != LF_F16 && out->dtype != LF_BF16 && out->dtype != LF_U8)
    return fail(LF_ERR_INVALID_ARG, "out dtype %d is not F32/F16/BF16/U8", out->dtype);
  if (out->n_chunk != 1 || out->width != g.nx || out->height != g.ny)
    return fail(LF_ERR_INVALID_ARG, "out must be one %dx%d plane", g.nx, g.ny);
  if (!out->rgba || !out->depth) return fail(LF_ERR_INVALID_ARG, "out rgba/depth is NULL");
  if (!workspace) return fail(LF_ERR_INVALID_ARG, "workspace is NULL");
  const int64_t n = field->n;
  const int64_t cap = capacity_of(field->kind, n, 1, g.wp, g.hp, workspace_bytes);
  if (cap < 1) return fail(LF_ERR_CAPACITY, "workspace of %zu bytes is too small for this field", workspace_bytes);
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  // Eq. 5: the view camera at (dx, dy, 0), principal point c + p N / 2 with p = d / (D_focal tan(theta / 2))
  const double px = (double)view->dx / ((double)cam->d_focal * g.tx);
  const double py = (double)view->dy / ((double)cam->d_focal * g.ty);
  g.c.t[0] = (float)((double)cam->t[0] - (double)view->dx);
  g.c.t[1] = (float)((double)cam->t[1] - (double)view->dy);
  g.c.cpx = (float)(g.cpx + px * g.nx / 2.0);
  g.c.cpy = (float)(g.cpy + py * g.ny / 2.0);
  const BuildLayout L = build_layout(field->kind, n, 1, g.wp, g.hp, cap);
  BuildArgs a;
  build_args(a, L, field, &vc, g, 1, LF_BIN_QUANTILE, out, workspace, cap);
  if ((e = build_planes(a, L, (hipStream_t)stream, &ctx->prof)) != hipSuccess) return hip_fail(e, "render launch");
  return LF_OK;
}

extern "C" lf_status lf_build_mpi_backward(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, const lf_mpi* mpi,
                                           const float* d_planes, const lf_gaussian_grads* grads, void* workspace,
                                           size_t workspace_bytes, void* stream) {
  if (!mpi) return fail(LF_ERR_INVALID_ARG, "mpi is NULL");
  Geom g;
  lf_status s = check_common(field, cam, mpi->n_chunk, &g);
  if (s != LF_OK) return s;
  if (field->kind != LF_GAUSSIANS) return fail(LF_ERR_UNSUPPORTED, "the build backward covers Gaussian fields only");
  if (mpi->width != g.wp || mpi->height != g.hp)
    return fail(LF_ERR_INVALID_ARG, "mpi is %dx%d but the camera's planes are %dx%d", mpi->width, mpi->height, g.wp,
                g.hp);
  if (!d_planes) return fail(LF_ERR_INVALID_ARG, "d_planes is NULL");
  if (!grads) return fail(LF_ERR_INVALID_ARG, "grads is NULL");
  if (field->n > 0 && !(grads->means && grads->log_scales && grads->quats && grads->opacity && grads->rgb))
    return fail(LF_ERR_INVALID_ARG, "a gradient output pointer is NULL");
  if (!workspace) return fail(LF_ERR_INVALID_ARG, "workspace is NULL");
  const int64_t cap = capacity_of(field->kind, field->n, mpi->n_chunk, g.wp, g.hp, workspace_bytes);
  if (cap < 1) return fail(LF_ERR_CAPACITY, "workspace of %zu bytes is too small for this field", workspace_bytes);
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const BuildLayout L = build_layout(field->kind, field->n, mpi->n_chunk, g.wp, g.hp, cap);
  if (L.tile_bits + L.chunk_bits > 32)
    return fail(LF_ERR_INVALID_ARG, "%d tiles x %d chunks do not fit a 32-bit (tile, chunk) key", L.n_tiles,
                mpi->n_chunk);
  BuildArgs a;
  build_args(a, L, field, cam, g, mpi->n_chunk, LF_BIN_QUANTILE, mpi, workspace, cap);
  // the forward left the tile-sorted entries in the array its radix passes ended on
  if (radix_passes(L.tile_bits, tile_digit_bits()) & 1) a.evals = a.evals_alt;
  a.d_planes = d_planes;
  a.grads = *grads;
  if ((e = build_backward(a, L, (hipStream_t)stream, &ctx->prof)) != hipSuccess) return hip_fail(e, "build backward launch");
  return LF_OK;
}

extern "C" lf_status lf_build_tile_lists(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, int32_t n_chunk,
                                         const void* workspace, size_t workspace_bytes, int32_t* tile, int32_t* tiles_x,
                                         int32_t* tiles_y, int64_t* bucket_start, int32_t* entries, void* stream) {
  Geom g;
  lf_status s = check_common(field, cam, n_chunk, &g);
  if (s != LF_OK) return s;
  if (!tile || !tiles_x || !tiles_y) return fail(LF_ERR_INVALID_ARG, "tile, tiles_x or tiles_y is NULL");
  if (!workspace) return fail(LF_ERR_INVALID_ARG, "workspace is NULL");
  const int64_t cap = capacity_of(field->kind, field->n, n_chunk, g.wp, g.hp, workspace_bytes);
  if (cap < 1) return fail(LF_ERR_CAPACITY, "workspace of %zu bytes is too small for this field", workspace_bytes);
  const BuildLayout L = build_layout(field->kind, field->n, n_chunk, g.wp, g.hp, cap);
  *tile = kTile;
  *tiles_x = L.ntx;
  *tiles_y = L.nty;
  if (!bucket_start && !entries) return LF_OK;
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  if (field->n == 0) return fail(LF_ERR_UNSUPPORTED, "an empty field has no tile lists");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  BuildArgs a;
  lf_mpi none{LF_F32, n_chunk, g.hp, g.wp, nullptr, nullptr, nullptr, nullptr};
  build_args(a, L, field, cam, g, n_chunk, LF_BIN_QUANTILE, &none, const_cast<void*>(workspace), cap);
  if (radix_passes(L.tile_bits, tile_digit_bits()) & 1) a.evals = a.evals_alt;
  if ((e = tile_lists_launch(a, L, bucket_start, entries, (hipStream_t)stream)) != hipSuccess)
    return hip_fail(e, "tile list copy");
  return LF_OK;
}

extern "C" lf_status lf_build_splat_work(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, int32_t n_chunk,
                                        const void* workspace, size_t workspace_bytes, int64_t* counts, void* stream) {
  Geom g;
  lf_status s = check_common(field, cam, n_chunk, &g);
  if (s != LF_OK) return s;
  if (field->kind != LF_GAUSSIANS) return fail(LF_ERR_UNSUPPORTED, "the splat work count covers Gaussian fields only");
  if (!counts) return fail(LF_ERR_INVALID_ARG, "counts is NULL");
  if (!workspace) return fail(LF_ERR_INVALID_ARG, "workspace is NULL");
  const int64_t cap = capacity_of(field->kind, field->n, n_chunk, g.wp, g.hp, workspace_bytes);
  if (cap < 1) return fail(LF_ERR_CAPACITY, "workspace of %zu bytes is too small for this field", workspace_bytes);
  const BuildLayout L = build_layout(field->kind, field->n, n_chunk, g.wp, g.hp, cap);
  if (L.tile_bits + L.chunk_bits > 32)
    return fail(LF_ERR_INVALID_ARG, "%d tiles x %d chunks do not fit a 32-bit (tile, chunk) key", L.n_tiles, n_chunk);
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  BuildArgs a;
  lf_mpi none{LF_F32, n_chunk, g.hp, g.wp, nullptr, nullptr, nullptr, nullptr};
  build_args(a, L, field, cam, g, n_chunk, LF_BIN_QUANTILE, &none, const_cast<void*>(workspace), cap);
  if (radix_passes(L.tile_bits, tile_digit_bits()) & 1) a.evals = a.evals_alt;
  if ((e = splat_work_launch(a, L, counts, (hipStream_t)stream)) != hipSuccess) return hip_fail(e, "splat work count");
  return LF_OK;
}

extern "C" lf_status lf_build_stats(lf_ctx* ctx, const void* workspace, size_t workspace_bytes, lf_build_info* out,
                                    void* stream) {
  if (!out) return fail(LF_ERR_INVALID_ARG, "out is NULL");
  if (!workspace || workspace_bytes < sizeof(BuildHeader)) return fail(LF_ERR_INVALID_ARG, "workspace is NULL or too small");
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  BuildHeader h;
  if ((e = hipMemcpyAsync(&h, workspace, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream)) != hipSuccess)
    return hip_fail(e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  out->n_visible = h.n_vis;
  out->entries_needed = h.entries;
  out->entry_capacity = h.capacity;
  out->overflow = h.overflow;
  out->stalled = h.stalled ? 1 : 0;
  if (h.stalled)
    return fail(LF_ERR_HIP, "a device-wide wait of the last build's sorts or scans timed out (planes are invalid)");
  if (h.overflow)
    return fail(LF_ERR_CAPACITY, "the last build needed %lld entries but the workspace holds %lld",
                (long long)h.entries, (long long)h.capacity);
  return LF_OK;
}
