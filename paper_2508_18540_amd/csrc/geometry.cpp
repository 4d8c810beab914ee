// Host geometry of the display and the reference camera (Sec. 4.2-4.3, Eqs. 1-5, 8),
// evaluated in double precision and rounded once to the float32 constants the kernels use.
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "lf_internal.h"

namespace lf {

static thread_local char g_err[512] = "";

lf_status fail(lf_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

lf_status hip_fail(hipError_t e, const char* what) {
  return fail(LF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err; }

static int round_half_up(double v) { return (int)std::floor(v + 0.5); }

static void split(double v, float* hi, float* lo) {
  *hi = (float)v;
  *lo = (float)(v - (double)*hi);
}

lf_status derive_geometry(const lf_camera* cam, Geom* g) {
  if (!cam) return fail(LF_ERR_INVALID_ARG, "camera is NULL");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(cam->R[i])) return fail(LF_ERR_INVALID_ARG, "camera R[%d] is not finite", i);
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(cam->t[i])) return fail(LF_ERR_INVALID_ARG, "camera t[%d] is not finite", i);
  if (cam->nx < 1 || cam->ny < 1 || cam->nx > LF_MAX_RES || cam->ny > LF_MAX_RES)
    return fail(LF_ERR_INVALID_ARG, "view resolution %dx%d outside [1, %d]", cam->nx, cam->ny, LF_MAX_RES);
  const double pi = 3.14159265358979323846;
  if (!(cam->fov_x > 0.0f && cam->fov_x < pi && cam->fov_y > 0.0f && cam->fov_y < pi))
    return fail(LF_ERR_INVALID_ARG, "field of view must lie in (0, pi)");
  if (!(cam->phi_x >= 0.0f && cam->phi_x < pi && cam->phi_y >= 0.0f && cam->phi_y < pi))
    return fail(LF_ERR_INVALID_ARG, "viewing angles must lie in [0, pi)");
  if (!(cam->d_focal > 0.0f) || !std::isfinite(cam->d_focal))
    return fail(LF_ERR_INVALID_ARG, "d_focal must be positive and finite");
  if (!(cam->d_shift >= 0.0f) || !std::isfinite(cam->d_shift))
    return fail(LF_ERR_INVALID_ARG, "d_shift must be >= 0 and finite");
  if (!(cam->z_near > 0.0f) || !std::isfinite(cam->z_near))
    return fail(LF_ERR_INVALID_ARG, "z_near must be positive and finite");
  if (!(cam->plane_scale > 0.0f) || !std::isfinite(cam->plane_scale))
    return fail(LF_ERR_INVALID_ARG, "plane_scale must be positive and finite");
  if (!(cam->dilation >= 0.0f) || !std::isfinite(cam->dilation))
    return fail(LF_ERR_INVALID_ARG, "dilation must be >= 0 and finite");

  const double Df = cam->d_focal;
  g->tx = std::tan(0.5 * (double)cam->fov_x);
  g->ty = std::tan(0.5 * (double)cam->fov_y);
  g->taux = std::tan(0.5 * (double)cam->phi_x);
  g->tauy = std::tan(0.5 * (double)cam->phi_y);
  // Eq. 1: forward shift covering both axes; Eq. 2: reference half-angle tangents.
  const double dx0 = Df * g->taux / (g->taux + g->tx);
  const double dy0 = Df * g->tauy / (g->tauy + g->ty);
  g->d_forward0 = dx0 > dy0 ? dx0 : dy0;
  g->tpx = Df * g->tx / (Df - g->d_forward0);
  g->tpy = Df * g->ty / (Df - g->d_forward0);
  g->d_forward = g->d_forward0 - (double)cam->d_shift;   // D_shift after theta' (Sec. 4.2)
  const double ps = cam->plane_scale;
  g->nx = cam->nx;
  g->ny = cam->ny;
  g->wp = round_half_up(ps * cam->nx);
  g->hp = round_half_up(ps * cam->ny);
  if (g->wp < 1 || g->hp < 1 || g->wp > LF_MAX_RES || g->hp > LF_MAX_RES)
    return fail(LF_ERR_INVALID_ARG, "plane resolution %dx%d outside [1, %d]", g->wp, g->hp, LF_MAX_RES);
  g->fx = 0.5 * cam->nx / g->tx;
  g->fy = 0.5 * cam->ny / g->ty;
  g->cx = 0.5 * (cam->nx - 1);
  g->cy = 0.5 * (cam->ny - 1);
  g->fpx = 0.5 * g->wp / g->tpx;
  g->fpy = 0.5 * g->hp / g->tpy;
  g->cpx = 0.5 * (g->wp - 1);
  g->cpy = 0.5 * (g->hp - 1);
  // Eq. 8: dilation aligned with the base camera's pixel size on the focal plane, unless
  // the camera asks for a constant one
  const double r = Df * g->tx / ((Df - g->d_forward) * g->tpx) * ps;
  g->f_dil = cam->dilation > 0.0f ? (double)cam->dilation : 0.3 * (r * r);

  Consts& c = g->c;
  split(g->d_forward, &c.d_fwd, &c.d_fwd_lo);
  c.z_near = cam->z_near;
  c.guard_x = (float)(1.3 * g->tpx);
  c.guard_y = (float)(1.3 * g->tpy);
  c.ratio_x = (float)((g->wp * g->tx) / (g->nx * g->tpx));
  c.ratio_y = (float)((g->hp * g->ty) / (g->ny * g->tpy));
  split(g->fpx, &c.fpx, &c.fpx_lo);
  split(g->fpy, &c.fpy, &c.fpy_lo);
  c.cpx = (float)g->cpx;
  c.cpy = (float)g->cpy;
  c.cx = (float)g->cx;
  c.cy = (float)g->cy;
  c.inv_focal = (float)(1.0 / Df);
  c.f_dil = (float)g->f_dil;
  for (int i = 0; i < 9; ++i) c.R[i] = cam->R[i];
  for (int i = 0; i < 3; ++i) c.t[i] = cam->t[i];
  c.nx = g->nx;
  c.ny = g->ny;
  c.wp = g->wp;
  c.hp = g->hp;
  return LF_OK;
}

}  // namespace lf

extern "C" const char* lf_last_error(void) { return lf::last_error(); }

extern "C" lf_status lf_geometry(const lf_camera* cam, lf_geometry_info* out) {
  if (!out) return lf::fail(LF_ERR_INVALID_ARG, "out is NULL");
  lf::Geom g;
  lf_status s = lf::derive_geometry(cam, &g);
  if (s != LF_OK) return s;
  out->d_forward0 = g.d_forward0;
  out->d_forward = g.d_forward;
  out->tan_half_theta_prime_x = g.tpx;
  out->tan_half_theta_prime_y = g.tpy;
  out->f_dilation = g.f_dil;
  out->fpx = g.fpx;
  out->fpy = g.fpy;
  out->cpx = g.cpx;
  out->cpy = g.cpy;
  out->fx = g.fx;
  out->fy = g.fy;
  out->cx = g.cx;
  out->cy = g.cy;
  out->plane_width = g.wp;
  out->plane_height = g.hp;
  out->d_forward32 = g.c.d_fwd;
  out->guard_x32 = g.c.guard_x;
  out->guard_y32 = g.c.guard_y;
  out->ratio_x32 = g.c.ratio_x;
  out->ratio_y32 = g.c.ratio_y;
  out->fpx32 = g.c.fpx;
  out->fpy32 = g.c.fpy;
  out->cpx32 = g.c.cpx;
  out->cpy32 = g.c.cpy;
  out->cx32 = g.c.cx;
  out->cy32 = g.c.cy;
  out->inv_focal32 = g.c.inv_focal;
  return LF_OK;
}

extern "C" lf_status lf_quilt_views(const lf_camera* cam, int32_t vx, int32_t vy, lf_view* out) {
  if (!out) return lf::fail(LF_ERR_INVALID_ARG, "out is NULL");
  if (vx < 1 || vy < 1 || (int64_t)vx * vy > 1 << 20)
    return lf::fail(LF_ERR_INVALID_ARG, "quilt %dx%d is empty or too large", vx, vy);
  lf::Geom g;
  lf_status s = lf::derive_geometry(cam, &g);
  if (s != LF_OK) return s;
  const double Df = cam->d_focal;
  for (int i = 0; i < vy; ++i) {
    // Eq. 3 (s = 0 for a single row), Eq. 4
    const double sy = vy > 1 ? (double)i / (vy - 1) - 0.5 : 0.0;
    for (int j = 0; j < vx; ++j) {
      const double sx = vx > 1 ? (double)j / (vx - 1) - 0.5 : 0.0;
      out[i * vx + j].dx = (float)(2.0 * Df * sx * g.taux);
      out[i * vx + j].dy = (float)(2.0 * Df * sy * g.tauy);
    }
  }
  return LF_OK;
}
