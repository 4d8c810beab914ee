// Spherical-harmonic colour for gfx950 (the SH ablation of Fig. 6): the swizzle blending of
// SH planes into views, and the colours of the Gaussians seen from one view.
//
// Composite of SH planes.  A plane texel holds the blended coefficients q_j (r, g, b) and
// A = 1 - T.  View v samples plane k at pixel (x, y) with the RGB composite's float32 texel
// program (Eq. 6, nearest or bilinear over all the texel's floats), and the sample adds the
// premultiplied colour max(sum_j q_j Y_j(d) + A / 2, 0), d the unit world direction of the
// pixel's ray (the same for every plane, so Y is evaluated once per pixel); Eq. 7 then
// blends the samples front to back.  One thread per output pixel; an SH texel is 16 to 208
// bytes, read straight from global memory.
#include "lf_internal.h"
#include "sh_basis.h"

namespace lf {
namespace {

template <int NC, bool BIL>
__global__ __launch_bounds__(256) void composite_sh(CompositeArgs a, ShView sv) {
  constexpr int TF = sh_texel_floats(NC);
  constexpr int T4 = TF / 4;
  const int64_t n = (int64_t)a.n_views * a.ny * a.nx;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % a.nx);
  const int y = (int)((i / a.nx) % a.ny);
  const int v = (int)(i / ((int64_t)a.nx * a.ny));
  const float4* planes = static_cast<const float4*>(a.planes);
  const float xr = (float)x - a.c.cx, yr = (float)y - a.c.cy;
  const float dx = a.dx[v], dy = a.dy[v];
  // the pixel's ray in view v (base-camera axes), then in world axes: R^T r
  const float rx = ((float)x - (a.c.cx + dx * sv.kx)) * sv.inv_fx;
  const float ry = ((float)y - (a.c.cy + dy * sv.ky)) * sv.inv_fy;
  const float* R = a.c.R;
  const float wx = R[0] * rx + R[3] * ry + R[6];
  const float wy = R[1] * rx + R[4] * ry + R[7];
  const float wz = R[2] * rx + R[5] * ry + R[8];
  const float inv = 1.0f / sqrtf(wx * wx + wy * wy + wz * wz);
  float Y[NC];
  sh_basis<NC>(wx * inv, wy * inv, wz * inv, Y);
  float Qr = 0.f, Qg = 0.f, Qb = 0.f, Tr = 1.f;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int k = 0; k < a.K; ++k) {
    const PlaneCo pc = plane_co(a.depth[k], a.c);
    const float cx = a.c.cpx + pc.gx * dx;
    const float cy = a.c.cpy + pc.gy * dy;
    const size_t base = (size_t)k * a.hp * a.wp;
    float f[TF];
    auto put = [&](int j, float4 v) {
      f[4 * j] = v.x;
      f[4 * j + 1] = v.y;
      f[4 * j + 2] = v.z;
      f[4 * j + 3] = v.w;
    };
    if (!BIL) {
      const float X = pc.bx * xr + (cx + 0.5f);
      const float Yc = pc.by * yr + (cy + 0.5f);
      const int ix = __float2int_rd(X), iy = __float2int_rd(Yc);
      const bool in = ix >= 0 && ix < a.wp && iy >= 0 && iy < a.hp;
      const float4* t = planes + (base + (size_t)(in ? iy : 0) * a.wp + (in ? ix : 0)) * T4;
#pragma unroll
      for (int j = 0; j < T4; ++j) put(j, in ? t[j] : z4);
    } else {
      const float X = pc.bx * xr + cx;
      const float Yc = pc.by * yr + cy;
      const float fx0 = floorf(X), fy0 = floorf(Yc);
      const float ax = X - fx0, ay = Yc - fy0;
      const int ix = __float2int_rd(fx0), iy = __float2int_rd(fy0);
      const float4* t[2][2];
      bool in[2][2];
#pragma unroll
      for (int oy = 0; oy < 2; ++oy)
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
          const int xx = ix + ox, yy = iy + oy;
          in[oy][ox] = xx >= 0 && xx < a.wp && yy >= 0 && yy < a.hp;
          t[oy][ox] = planes + (base + (size_t)(in[oy][ox] ? yy : 0) * a.wp + (in[oy][ox] ? xx : 0)) * T4;
        }
#pragma unroll
      for (int j = 0; j < T4; ++j) {
        const float4 t00 = in[0][0] ? t[0][0][j] : z4, t01 = in[0][1] ? t[0][1][j] : z4;
        const float4 t10 = in[1][0] ? t[1][0][j] : z4, t11 = in[1][1] ? t[1][1][j] : z4;
        const float4 r0 = make_float4(fmaf(ax, t01.x - t00.x, t00.x), fmaf(ax, t01.y - t00.y, t00.y),
                                      fmaf(ax, t01.z - t00.z, t00.z), fmaf(ax, t01.w - t00.w, t00.w));
        const float4 r1 = make_float4(fmaf(ax, t11.x - t10.x, t10.x), fmaf(ax, t11.y - t10.y, t10.y),
                                      fmaf(ax, t11.z - t10.z, t10.z), fmaf(ax, t11.w - t10.w, t10.w));
        put(j, make_float4(fmaf(ay, r1.x - r0.x, r0.x), fmaf(ay, r1.y - r0.y, r0.y), fmaf(ay, r1.z - r0.z, r0.z),
                           fmaf(ay, r1.w - r0.w, r0.w)));
      }
    }
    const float A = f[3];
    float cr = fmaf(f[0], Y[0], 0.5f * A), cg = fmaf(f[1], Y[0], 0.5f * A), cb = fmaf(f[2], Y[0], 0.5f * A);
#pragma unroll
    for (int j = 1; j < NC; ++j) {
      cr = fmaf(f[4 + 3 * (j - 1)], Y[j], cr);
      cg = fmaf(f[5 + 3 * (j - 1)], Y[j], cg);
      cb = fmaf(f[6 + 3 * (j - 1)], Y[j], cb);
    }
    Qr = fmaf(Tr, fmaxf(cr, 0.0f), Qr);
    Qg = fmaf(Tr, fmaxf(cg, 0.0f), Qg);
    Qb = fmaf(Tr, fmaxf(cb, 0.0f), Qb);
    Tr = fmaf(-Tr, A, Tr);
  }
  reinterpret_cast<float4*>(a.out)[i] = make_float4(Qr, Qg, Qb, Tr);
}

template <int NC>
__global__ __launch_bounds__(256) void sh_colours(const float* __restrict__ means, const float* __restrict__ sh,
                                                  int64_t n, float cx, float cy, float cz, float* __restrict__ rgb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float dx = means[3 * i] - cx, dy = means[3 * i + 1] - cy, dz = means[3 * i + 2] - cz;
  const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  float Y[NC];
  sh_basis<NC>(dx * inv, dy * inv, dz * inv, Y);
  const float* c = sh + (size_t)i * 3 * NC;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float v = 0.5f;
#pragma unroll
    for (int j = 0; j < NC; ++j) v = fmaf(c[3 * j + ch], Y[j], v);
    rgb[3 * i + ch] = fmaxf(v, 0.0f);
  }
}

template <int NC>
hipError_t launch_composite(const CompositeArgs& a, const ShView& sv, hipStream_t s) {
  const int64_t n = (int64_t)a.n_views * a.ny * a.nx;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (a.interp == LF_BILINEAR) hipLaunchKernelGGL((composite_sh<NC, true>), grid, dim3(256), 0, s, a, sv);
  else hipLaunchKernelGGL((composite_sh<NC, false>), grid, dim3(256), 0, s, a, sv);
  return hipGetLastError();
}

}  // namespace

hipError_t composite_sh_launch(const CompositeArgs& a, int n_coef, const ShView& sv, hipStream_t s) {
  switch (n_coef) {
    case 1: return launch_composite<1>(a, sv, s);
    case 4: return launch_composite<4>(a, sv, s);
    case 9: return launch_composite<9>(a, sv, s);
    default: return launch_composite<16>(a, sv, s);
  }
}

hipError_t sh_colours_launch(const float* means, const float* sh, int n_coef, int64_t n, const float centre[3],
                             float* rgb, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256));
  const float cx = centre[0], cy = centre[1], cz = centre[2];
  switch (n_coef) {
    case 1: hipLaunchKernelGGL((sh_colours<1>), grid, dim3(256), 0, s, means, sh, n, cx, cy, cz, rgb); break;
    case 4: hipLaunchKernelGGL((sh_colours<4>), grid, dim3(256), 0, s, means, sh, n, cx, cy, cz, rgb); break;
    case 9: hipLaunchKernelGGL((sh_colours<9>), grid, dim3(256), 0, s, means, sh, n, cx, cy, cz, rgb); break;
    default: hipLaunchKernelGGL((sh_colours<16>), grid, dim3(256), 0, s, means, sh, n, cx, cy, cz, rgb); break;
  }
  return hipGetLastError();
}

}  // namespace lf
