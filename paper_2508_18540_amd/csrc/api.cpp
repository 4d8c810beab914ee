// C ABI entry points: argument validation on the host, then kernel launches.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "lf_internal.h"
#include "sh_basis.h"

namespace lf {
namespace {

bool dtype_ok(int32_t d) { return d == LF_F32 || d == LF_F16 || d == LF_BF16 || d == LF_U8; }

lf_status check_mpi(const lf_mpi* mpi, const Geom& g) {
  if (!mpi) return fail(LF_ERR_INVALID_ARG, "mpi is NULL");
  if (!dtype_ok(mpi->dtype)) return fail(LF_ERR_INVALID_ARG, "mpi dtype %d is not F32/F16/BF16/U8", mpi->dtype);
  if (mpi->n_chunk < 1 || mpi->n_chunk > LF_MAX_CHUNKS)
    return fail(LF_ERR_INVALID_ARG, "n_chunk %d outside [1, %d]", mpi->n_chunk, LF_MAX_CHUNKS);
  if (mpi->width != g.wp || mpi->height != g.hp)
    return fail(LF_ERR_INVALID_ARG, "mpi is %dx%d but the camera's planes are %dx%d", mpi->width, mpi->height,
                g.wp, g.hp);
  if (!mpi->rgba || !mpi->depth) return fail(LF_ERR_INVALID_ARG, "mpi rgba/depth is NULL");
  return LF_OK;
}

lf_status check_views(const lf_view* views, int32_t n_views) {
  if (!views) return fail(LF_ERR_INVALID_ARG, "views is NULL");
  if (n_views < 1 || n_views > LF_MAX_VIEWS)
    return fail(LF_ERR_INVALID_ARG, "n_views %d outside [1, %d]", n_views, LF_MAX_VIEWS);
  for (int v = 0; v < n_views; ++v)
    if (!std::isfinite(views[v].dx) || !std::isfinite(views[v].dy))
      return fail(LF_ERR_INVALID_ARG, "view %d offset is not finite", v);
  return LF_OK;
}

}  // namespace

lf_status composite_args(const lf_mpi* mpi, const lf_camera* cam, const lf_view* views, int32_t n_views,
                         CompositeArgs* a) {
  Geom g;
  lf_status s = derive_geometry(cam, &g);
  if (s != LF_OK) return s;
  if ((s = check_mpi(mpi, g)) != LF_OK) return s;
  if ((s = check_views(views, n_views)) != LF_OK) return s;
  std::memset(a, 0, sizeof(*a));
  a->planes = mpi->rgba;
  a->depth = mpi->depth;
  a->K = mpi->n_chunk;
  a->hp = g.hp;
  a->wp = g.wp;
  a->nx = g.nx;
  a->ny = g.ny;
  a->n_views = n_views;
  a->plane_dtype = mpi->dtype;
  a->c = g.c;
  for (int v = 0; v < n_views; ++v) {
    a->dx[v] = views[v].dx;
    a->dy[v] = views[v].dy;
  }
  return LF_OK;
}

namespace {

lf_status check_ctx(lf_ctx* ctx) {
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return LF_OK;
}

}  // namespace
}  // namespace lf

using namespace lf;

// Device memory of lf_composite_noalloc's coefficient table: a file-scope array every GPU
// the library runs on holds until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol); it uses the device
// address lf_create resolves once per device with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[LF_COMPOSITE_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
void* scratch_ptr[kMaxDevices] = {};

// Resolves this device's address of `scratch` (the device must be current); once per device.
hipError_t resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) scratch_ptr[device] = p;
  return e;
}

}  // namespace

extern "C" const char* lf_version(void) { return "lf-mi355x 0.1 (gfx950)"; }

extern "C" lf_status lf_create(lf_ctx** out, int device) {
  if (!out) return fail(LF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(LF_ERR_HIP, "no HIP device available");
  if (device < 0 || device >= n) return fail(LF_ERR_INVALID_ARG, "device %d outside [0, %d)", device, n);
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  lf_ctx* c = new (std::nothrow) lf_ctx;
  if (!c) return fail(LF_ERR_OUT_OF_MEMORY, "context allocation failed");
  c->device = device;
  // The composite's coefficient table, sized once for the largest call (LF_MAX_CHUNKS planes,
  // LF_MAX_VIEWS views, about 21 MB): lf_composite and lf_composite_backward then never
  // allocate, free or synchronise, so they can be captured into a graph, and a captured
  // graph's table stays valid until lf_destroy.
  c->table_bytes = composite_table_bytes(LF_MAX_CHUNKS, LF_MAX_VIEWS);
  if ((e = hipMalloc(&c->table, c->table_bytes)) != hipSuccess) {
    delete c;
    return hip_fail(e, "composite coefficient table");
  }
  if ((e = resolve_scratch(device)) != hipSuccess) {
    hipFree(c->table);
    delete c;
    return hip_fail(e, "hipGetSymbolAddress of the composite scratch table");
  }
  *out = c;
  return LF_OK;
}

extern "C" void lf_destroy(lf_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  ctx->prof.release();
  if (ctx->table) hipFree(ctx->table);
  delete ctx;
}

namespace lf {

hipEvent_t Profiler::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing only: no system-scope fence (cache write-back and invalidation) when an event is
  // recorded; with it, each phase boundary cost about 4 us and cooled the caches of the
  // phase after it
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

size_t Profiler::begin(int phase, hipStream_t s) {
  Rec r{phase, take(), take()};
  if (r.a) hipEventRecord(r.a, s);
  recs.push_back(r);
  return recs.size() - 1;
}

void Profiler::end(size_t rec, hipStream_t s) {
  if (rec < recs.size() && recs[rec].b) hipEventRecord(recs[rec].b, s);
}

hipError_t Profiler::collect() {
  hipError_t err = hipSuccess;
  for (Rec& r : recs) {
    if (r.a && r.b) {
      hipError_t e = hipEventSynchronize(r.b);
      float t = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
      if (e == hipSuccess) {
        ms[r.phase] += t;
        count[r.phase] += 1;
      } else {
        err = e;
      }
    }
    if (r.a) pool.push_back(r.a);
    if (r.b) pool.push_back(r.b);
  }
  recs.clear();
  return err;
}

void Profiler::release() {
  collect();
  for (hipEvent_t e : pool) hipEventDestroy(e);
  pool.clear();
}

}  // namespace lf

extern "C" lf_status lf_profile_enable(lf_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  ctx->prof.on = enable != 0;
  return LF_OK;
}

extern "C" lf_status lf_profile_read(lf_ctx* ctx, double* ms, int64_t* count, int32_t reset) {
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  if (!ms || !count) return fail(LF_ERR_INVALID_ARG, "ms/count is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  e = ctx->prof.collect();
  for (int i = 0; i < LF_NUM_PHASES; ++i) {
    ms[i] = ctx->prof.ms[i];
    count[i] = ctx->prof.count[i];
    if (reset) {
      ctx->prof.ms[i] = 0.0;
      ctx->prof.count[i] = 0;
    }
  }
  if (e != hipSuccess) return hip_fail(e, "profiling events");
  return LF_OK;
}

extern "C" lf_status lf_composite(lf_ctx* ctx, const lf_mpi* mpi, const lf_camera* cam, const lf_view* views,
                                  int32_t n_views, int32_t interp, int32_t out_dtype, void* out, void* stream) {
  CompositeArgs* a = new (std::nothrow) CompositeArgs;
  if (!a) return fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
  lf_status s = composite_args(mpi, cam, views, n_views, a);
  if (s == LF_OK && interp != LF_NEAREST && interp != LF_BILINEAR)
    s = fail(LF_ERR_INVALID_ARG, "interp %d is not NEAREST/BILINEAR", interp);
  if (s == LF_OK && out_dtype != LF_F32 && out_dtype != LF_F16)
    s = fail(LF_ERR_INVALID_ARG, "out_dtype %d is not F32/F16", out_dtype);
  if (s == LF_OK && !out) s = fail(LF_ERR_INVALID_ARG, "out is NULL");
  if (s == LF_OK) s = check_ctx(ctx);
  if (s == LF_OK) {
    a->interp = interp;
    a->out_dtype = out_dtype;
    a->out = out;
    const hipError_t e = composite_launch(*a, ctx->table, (hipStream_t)stream, &ctx->prof);
    if (e != hipSuccess) s = hip_fail(e, "composite launch");
  }
  delete a;
  return s;
}

extern "C" lf_status lf_composite_noalloc(lf_ctx* ctx, const lf_mpi* mpi, const lf_camera* cam,
                                          const lf_view* views, int32_t n_views, int32_t interp,
                                          int32_t out_dtype, void* out, void* stream) {
  // lf_composite with its table in the device's `scratch` array: no allocation of any kind
  // (the argument block lives on the stack, profiling is not used)
  CompositeArgs a;
  lf_status s = composite_args(mpi, cam, views, n_views, &a);
  if (s != LF_OK) return s;
  if (interp != LF_NEAREST && interp != LF_BILINEAR)
    return fail(LF_ERR_INVALID_ARG, "interp %d is not NEAREST/BILINEAR", interp);
  if (out_dtype != LF_F32 && out_dtype != LF_F16) return fail(LF_ERR_INVALID_ARG, "out_dtype %d is not F32/F16", out_dtype);
  if (!out) return fail(LF_ERR_INVALID_ARG, "out is NULL");
  const size_t need = composite_table_bytes(a.K, a.n_views);
  if (need > (size_t)LF_COMPOSITE_SCRATCH_BYTES)
    return fail(LF_ERR_CAPACITY, "%d planes x %d views need a %zu-byte coefficient table; the static scratch holds %zu",
                a.K, a.n_views, need, (size_t)LF_COMPOSITE_SCRATCH_BYTES);
  if ((s = check_ctx(ctx)) != LF_OK) return s;
  void* table = (ctx->device >= 0 && ctx->device < kMaxDevices) ? scratch_ptr[ctx->device] : nullptr;
  if (!table) return fail(LF_ERR_HIP, "the composite scratch table of device %d was not resolved", ctx->device);
  a.interp = interp;
  a.out_dtype = out_dtype;
  a.out = out;
  const hipError_t e = composite_launch(a, table, (hipStream_t)stream, nullptr);
  return e == hipSuccess ? LF_OK : hip_fail(e, "composite launch");
}

extern "C" lf_status lf_composite_backward(lf_ctx* ctx, const lf_mpi* mpi, const lf_camera* cam, const lf_view* views,
                                           int32_t n_views, int32_t interp, const float* d_out, float* d_planes,
                                           void* stream) {
  CompositeArgs* a = new (std::nothrow) CompositeArgs;
  if (!a) return fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
  lf_status s = composite_args(mpi, cam, views, n_views, a);
  if (s == LF_OK && interp != LF_NEAREST && interp != LF_BILINEAR)
    s = fail(LF_ERR_INVALID_ARG, "interp %d is not NEAREST/BILINEAR", interp);
  if (s == LF_OK && a->plane_dtype == LF_U8)
    s = fail(LF_ERR_UNSUPPORTED, "UNORM8 planes have no composite backward (the quantisation has no gradient)");
  if (s == LF_OK && !d_out) s = fail(LF_ERR_INVALID_ARG, "d_out is NULL");
  if (s == LF_OK && !d_planes) s = fail(LF_ERR_INVALID_ARG, "d_planes is NULL");
  if (s == LF_OK) s = check_ctx(ctx);
  if (s == LF_OK) {
    a->interp = interp;
    const hipError_t e = composite_backward_launch(*a, ctx->table, d_out, d_planes, (hipStream_t)stream, &ctx->prof);
    if (e != hipSuccess) s = hip_fail(e, "composite backward launch");
  }
  delete a;
  return s;
}

extern "C" int32_t lf_sh_texel_floats(int32_t degree) {
  if (degree < 0 || degree > LF_MAX_SH_DEGREE) return 0;
  return sh_texel_floats((degree + 1) * (degree + 1));
}

extern "C" lf_status lf_composite_sh(lf_ctx* ctx, const lf_sh_mpi* mpi, const lf_camera* cam, const lf_view* views,
                                     int32_t n_views, int32_t interp, float* out, void* stream) {
  if (!mpi) return fail(LF_ERR_INVALID_ARG, "mpi is NULL");
  if (mpi->degree < 0 || mpi->degree > LF_MAX_SH_DEGREE)
    return fail(LF_ERR_INVALID_ARG, "SH degree %d outside [0, %d]", mpi->degree, LF_MAX_SH_DEGREE);
  if (interp != LF_NEAREST && interp != LF_BILINEAR)
    return fail(LF_ERR_INVALID_ARG, "interp %d is not NEAREST/BILINEAR", interp);
  if (!out) return fail(LF_ERR_INVALID_ARG, "out is NULL");
  // the RGB composite's argument block over the SH texels (its dtype check sees F32)
  const lf_mpi m{LF_F32, mpi->n_chunk, mpi->height, mpi->width, mpi->planes, mpi->depth, nullptr, nullptr};
  CompositeArgs* a = new (std::nothrow) CompositeArgs;
  if (!a) return fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
  lf_status s = composite_args(&m, cam, views, n_views, a);
  Geom g;
  if (s == LF_OK) s = derive_geometry(cam, &g);
  if (s == LF_OK) s = check_ctx(ctx);
  if (s == LF_OK) {
    a->interp = interp;
    a->out_dtype = LF_F32;
    a->out = out;
    // Eq. 5: principal point c + p N / 2 with p = d / (D_focal tan(theta / 2))
    ShView sv;
    sv.kx = (float)((double)g.nx / (2.0 * (double)cam->d_focal * g.tx));
    sv.ky = (float)((double)g.ny / (2.0 * (double)cam->d_focal * g.ty));
    sv.inv_fx = (float)(1.0 / g.fx);
    sv.inv_fy = (float)(1.0 / g.fy);
    const int nc = (mpi->degree + 1) * (mpi->degree + 1);
    hipError_t e;
    {
      PhaseScope ps(&ctx->prof, LF_PHASE_COMPOSITE, (hipStream_t)stream);
      e = composite_sh_launch(*a, nc, sv, (hipStream_t)stream);
    }
    if (e != hipSuccess) s = hip_fail(e, "SH composite launch");
  }
  delete a;
  return s;
}

extern "C" lf_status lf_sh_colours(lf_ctx* ctx, const float* means, const float* sh, int32_t degree, int64_t n,
                                   const lf_camera* cam, const lf_view* view, float* rgb_out, void* stream) {
  if (degree < 0 || degree > LF_MAX_SH_DEGREE)
    return fail(LF_ERR_INVALID_ARG, "SH degree %d outside [0, %d]", degree, LF_MAX_SH_DEGREE);
  if (n < 0) return fail(LF_ERR_INVALID_ARG, "n is negative");
  if (n > 0 && !(means && sh && rgb_out)) return fail(LF_ERR_INVALID_ARG, "means, sh or rgb_out is NULL");
  if (!cam) return fail(LF_ERR_INVALID_ARG, "camera is NULL");
  if (!view) return fail(LF_ERR_INVALID_ARG, "view is NULL");
  if (!(std::isfinite(view->dx) && std::isfinite(view->dy))) return fail(LF_ERR_INVALID_ARG, "view offset is not finite");
  lf_status s = check_ctx(ctx);
  if (s != LF_OK) return s;
  // centre = R^T ((dx, dy, 0) - t)
  const double o[3] = {(double)view->dx - cam->t[0], (double)view->dy - cam->t[1], -(double)cam->t[2]};
  float centre[3];
  for (int i = 0; i < 3; ++i)
    centre[i] = (float)((double)cam->R[i] * o[0] + (double)cam->R[3 + i] * o[1] + (double)cam->R[6 + i] * o[2]);
  const hipError_t e = sh_colours_launch(means, sh, (degree + 1) * (degree + 1), n, centre, rgb_out, (hipStream_t)stream);
  return e == hipSuccess ? LF_OK : hip_fail(e, "SH colour launch");
}

extern "C" lf_status lf_plane_coeffs(lf_ctx* ctx, const lf_mpi* mpi, const lf_camera* cam, const lf_view* views,
                                     int32_t n_views, float* bx, float* by, float* cx, float* cy, float* cxn,
                                     float* cyn, void* stream) {
  CompositeArgs* a = new (std::nothrow) CompositeArgs;
  if (!a) return fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
  lf_status s = composite_args(mpi, cam, views, n_views, a);
  if (s == LF_OK && !(bx && by && cx && cy && cxn && cyn)) s = fail(LF_ERR_INVALID_ARG, "an output is NULL");
  if (s == LF_OK) s = check_ctx(ctx);
  if (s == LF_OK) {
    hipError_t e = plane_coeffs_launch(*a, bx, by, cx, cy, cxn, cyn, (hipStream_t)stream);
    if (e != hipSuccess) s = hip_fail(e, "plane_coeffs launch");
  }
  delete a;
  return s;
}
