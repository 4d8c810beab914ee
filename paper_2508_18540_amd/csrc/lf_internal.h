// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lf.h"

// Library context: the device it was created on.
struct lf_ctx {
  int device;
};

namespace lf {

// Float32 constants of the decision programs and of the projection.  The host derives
// every value in float64 (Eqs. 1-2, 8) and rounds it once; *_lo members hold the
// rounding residual (value - hi) so kernels can form double-float products.
struct Consts {
  float d_fwd, d_fwd_lo;     // reference camera position on the base camera's +z axis
  float z_near;
  float guard_x, guard_y;    // fl32(1.3 tan(theta'/2))
  float ratio_x, ratio_y;    // fl32(f'/f): plane texels per view pixel at unit magnification
  float fpx, fpx_lo, fpy, fpy_lo;   // reference focal lengths in texels
  float cpx, cpy;            // reference principal point (W_p - 1)/2, (H_p - 1)/2
  float cx, cy;              // view principal point (N - 1)/2
  float inv_focal;           // fl32(1 / D_focal)
  float f_dil;               // Eq. 8 dilation, texels^2
  float R[9], t[3];          // world -> base camera
  int32_t nx, ny, wp, hp;
};

struct Geom {
  double tx, ty, taux, tauy, d_forward0, d_forward, tpx, tpy;
  double fx, fy, cx, cy, fpx, fpy, cpx, cpy, f_dil;
  int32_t nx, ny, wp, hp;
  Consts c;
};

// Validates `cam` and derives its geometry.  Sets the thread's error message on failure.
lf_status derive_geometry(const lf_camera* cam, Geom* g);

// Thread-local error message helpers.
lf_status fail(lf_status s, const char* fmt, ...);
lf_status hip_fail(hipError_t e, const char* what);

struct CompositeArgs {
  const void* planes;
  const float* depth;
  void* out;
  int32_t K, hp, wp, nx, ny, n_views;
  int32_t plane_dtype, out_dtype, interp;
  Consts c;
  float dx[LF_MAX_VIEWS];
  float dy[LF_MAX_VIEWS];
};

hipError_t composite_launch(const CompositeArgs& a, hipStream_t s);
hipError_t plane_coeffs_launch(const CompositeArgs& a, float* bx, float* by, float* cx, float* cy,
                               float* cxn, float* cyn, hipStream_t s);

}  // namespace lf
