// Spherical-harmonic colour for gfx950 (the SH ablation of Fig. 6): the swizzle blending of
// SH planes into views, and the colours of the Gaussians seen from one view.
//
// Composite of SH planes.  A plane texel holds the blended coefficients q_j (r, g, b) and
// A = 1 - T.  View v samples plane k at pixel (x, y) with the RGB composite's float32 texel
// program (Eq. 6, nearest or bilinear over all the texel's floats), and the sample adds the
// premultiplied colour max(sum_j q_j Y_j(d) + A / 2, 0), d the unit world direction of the
// pixel's ray (the same for every plane, so Y is evaluated once per pixel); Eq. 7 then
// blends the samples front to back.  An SH texel is 16 to 208 bytes.  The row kernel below
// stages plane rows in LDS for a group of views; the per-pixel kernel (one thread per
// output pixel, texels read from global memory) is kept as the plain form.
#include <cstdlib>
#include <cstring>
#include <type_traits>

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

// Row kernel.  Views are grouped by dy (runs of kShGroup views of one class).  A work-group
// of four waves owns kShSeg pixels of one output row (one pixel per lane) for one group;
// wave w computes views w and w + 4 of the group.  Per plane the work-group stages into LDS
// the texels of the plane row that its samples reach (bilinear: the two rows blended
// vertically), so a texel is fetched once per work-group and read from LDS by every view
// of the group; a window longer than the buffer falls back to global reads for that plane.
// The LDS buffer is sized for three work-groups per CU.  The groups of a row share its
// plane rows, so the logical tiles (group fastest, then row segment, then row) are dealt to
// the 8 XCDs in contiguous runs (work-group w runs on XCD w mod 8) and meet in one L2.
constexpr int kShSeg = 64;
constexpr int kShWaves = 4;
constexpr int kShGroup = 8;
constexpr int kShWinBytes = 53248;

// Adds float f (index in the texel) of a sample to the colour sums; q_0 and A (floats 0-3)
// are taken first, floats past q_{NC-1} are padding.
template <int NC>
__device__ __forceinline__ void sh_add(int f, float v, const float* Y, float& cr, float& cg, float& cb) {
  if (f < 4 || f >= 4 + 3 * (NC - 1)) return;
  const int j = 1 + (f - 4) / 3, ch = (f - 4) % 3;
  if (ch == 0) cr = fmaf(v, Y[j], cr);
  else if (ch == 1) cg = fmaf(v, Y[j], cg);
  else cb = fmaf(v, Y[j], cb);
}

template <int NC, bool BIL>
__global__ __launch_bounds__(kShSeg * kShWaves) void composite_sh_rows(CompositeArgs a, ShView sv, int nseg,
                                                                       int total) {
  constexpr int TF = sh_texel_floats(NC);
  constexpr int T4 = TF / 4;
  constexpr int VW = kShGroup / kShWaves;                  // views per wave
  constexpr int WCAP = kShWinBytes / (TF * 4);
  constexpr int NT = kShSeg * kShWaves;
  extern __shared__ float4 win[];                          // WCAP texels of T4 float4
  const int w = blockIdx.x;
  const int per = (total + 7) / 8;
  const int lg = (w % 8) * per + w / 8;
  if (lg >= total) return;
  const int gi = lg % a.n_groups, rest = lg / a.n_groups;
  const int seg = rest % nseg, y = rest / nseg;
  const uint32_t gd = a.vgroup[gi];
  const int v0 = gd & 0xffu, nv = gd >> 8;
  const int tid = threadIdx.x, lane = tid & (kShSeg - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kShSeg);
  const int xs0 = seg * kShSeg, x = xs0 + lane;
  const int xs1 = min(xs0 + kShSeg, a.nx) - 1;
  const float xr = (float)x - a.c.cx, yr = (float)y - a.c.cy;
  const float xr_lo = (float)xs0 - a.c.cx, xr_hi = (float)xs1 - a.c.cx;
  const float dy = a.dy[a.perm[v0]];
  const float* R = a.c.R;
  // this wave's views (slot wave + kShWaves jj of the group)
  float dxv[VW], Yb[VW][NC], Qr[VW], Qg[VW], Qb[VW], Tr[VW];
#pragma unroll
  for (int jj = 0; jj < VW; ++jj) {
    dxv[jj] = a.dx[a.perm[v0 + min(wave + kShWaves * jj, nv - 1)]];
    const float rx = ((float)x - (a.c.cx + dxv[jj] * sv.kx)) * sv.inv_fx;
    const float ry = ((float)y - (a.c.cy + dy * sv.ky)) * sv.inv_fy;
    const float wx = R[0] * rx + R[3] * ry + R[6];
    const float wy = R[1] * rx + R[4] * ry + R[7];
    const float wz = R[2] * rx + R[5] * ry + R[8];
    const float inv = 1.0f / sqrtf(wx * wx + wy * wy + wz * wz);
    sh_basis<NC>(wx * inv, wy * inv, wz * inv, Yb[jj]);
    Qr[jj] = Qg[jj] = Qb[jj] = 0.0f;
    Tr[jj] = 1.0f;
  }
  const float4* planes = static_cast<const float4*>(a.planes);
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int k = 0; k < a.K; ++k) {
    const PlaneCo pc = plane_co(a.depth[k], a.c);
    const float cy = a.c.cpy + pc.gy * dy;
    int iy;
    float wyb = 0.0f;
    if (!BIL) {
      iy = __float2int_rd(pc.by * yr + (cy + 0.5f));
    } else {
      const float Yc = pc.by * yr + cy;
      const float fy0 = floorf(Yc);
      wyb = Yc - fy0;
      iy = __float2int_rd(fy0);
    }
    const bool r0ok = iy >= 0 && iy < a.hp, r1ok = BIL && iy + 1 >= 0 && iy + 1 < a.hp;
    if (!r0ok && !r1ok) continue;                          // the row misses the plane: no sample
    // window of the group's samples: X is monotone in x and in the view offset
    float cmin = 0.0f, cmax = 0.0f;
    for (int j = 0; j < nv; ++j) {
      const float cx = a.c.cpx + pc.gx * a.dx[a.perm[v0 + j]];
      const float cn = BIL ? cx : cx + 0.5f;
      cmin = j ? fminf(cmin, cn) : cn;
      cmax = j ? fmaxf(cmax, cn) : cn;
    }
    const float lo = floorf(pc.bx * xr_lo + cmin);
    const float hi = floorf(pc.bx * xr_hi + cmax) + (BIL ? 1.0f : 0.0f);
    const bool fits = lo >= -1.0e9f && hi <= 1.0e9f && hi >= lo && hi - lo + 1.0f <= (float)WCAP;
    const int f0 = fits ? (int)lo : 0, len = fits ? (int)(hi - lo) + 1 : 0;
    const size_t rb0 = ((size_t)k * a.hp + (r0ok ? iy : 0)) * a.wp;
    const size_t rb1 = ((size_t)k * a.hp + (r1ok ? iy + 1 : 0)) * a.wp;
    // vertically blended texel ix, float4 c, from global memory (zero outside the plane)
    auto fetch = [&](int ix, int c) -> float4 {
      const bool xin = ix >= 0 && ix < a.wp;
      const int cx = xin ? ix : 0;
      float4 t0 = (xin && r0ok) ? planes[(rb0 + cx) * T4 + c] : z4;
      if (BIL) {
        const float4 t1 = (xin && r1ok) ? planes[(rb1 + cx) * T4 + c] : z4;
        t0 = make_float4(fmaf(wyb, t1.x - t0.x, t0.x), fmaf(wyb, t1.y - t0.y, t0.y), fmaf(wyb, t1.z - t0.z, t0.z),
                         fmaf(wyb, t1.w - t0.w, t0.w));
      }
      return t0;
    };
    __syncthreads();                                       // the previous plane's window is consumed
    if (fits)
      for (int i = tid; i < len * T4; i += NT) win[i] = fetch(f0 + i / T4, i % T4);
    __syncthreads();
    // one view's sample: texels from the LDS window (FROM_LDS) or from global memory
    auto blend_view = [&](int jj, auto from_lds_tag) {
      constexpr bool FROM_LDS = decltype(from_lds_tag)::value;
      const float cx = a.c.cpx + pc.gx * dxv[jj];
      const float X = pc.bx * xr + (BIL ? cx : cx + 0.5f);
      int ix;
      float ax = 0.0f;
      if (!BIL) {
        ix = __float2int_rd(X);
      } else {
        const float fx0 = floorf(X);
        ax = X - fx0;
        ix = __float2int_rd(fx0);
      }
      // window slots of the sample's texels, computed once (clamped: lanes past the row end)
      const int w0 = FROM_LDS ? min(max(ix - f0, 0), len - 1) * T4 : 0;
      const int w1 = FROM_LDS && BIL ? min(max(ix + 1 - f0, 0), len - 1) * T4 : 0;
      auto sample = [&](int c) -> float4 {
        const float4 t0 = FROM_LDS ? win[w0 + c] : fetch(ix, c);
        if (!BIL) return t0;
        const float4 t1 = FROM_LDS ? win[w1 + c] : fetch(ix + 1, c);
        return make_float4(fmaf(ax, t1.x - t0.x, t0.x), fmaf(ax, t1.y - t0.y, t0.y), fmaf(ax, t1.z - t0.z, t0.z),
                           fmaf(ax, t1.w - t0.w, t0.w));
      };
      const float4 s0 = sample(0);
      const float A = s0.w;
      float cr = fmaf(s0.x, Yb[jj][0], 0.5f * A), cg = fmaf(s0.y, Yb[jj][0], 0.5f * A),
            cb = fmaf(s0.z, Yb[jj][0], 0.5f * A);
#pragma unroll
      for (int c = 1; c < T4; ++c) {
        const float4 sc = sample(c);
        sh_add<NC>(4 * c, sc.x, Yb[jj], cr, cg, cb);
        sh_add<NC>(4 * c + 1, sc.y, Yb[jj], cr, cg, cb);
        sh_add<NC>(4 * c + 2, sc.z, Yb[jj], cr, cg, cb);
        sh_add<NC>(4 * c + 3, sc.w, Yb[jj], cr, cg, cb);
      }
      Qr[jj] = fmaf(Tr[jj], fmaxf(cr, 0.0f), Qr[jj]);
      Qg[jj] = fmaf(Tr[jj], fmaxf(cg, 0.0f), Qg[jj]);
      Qb[jj] = fmaf(Tr[jj], fmaxf(cb, 0.0f), Qb[jj]);
      Tr[jj] = fmaf(-Tr[jj], A, Tr[jj]);
    };
    if (fits) {                                            // uniform: one straight path each
#pragma unroll
      for (int jj = 0; jj < VW; ++jj)
        if (wave + kShWaves * jj < nv) blend_view(jj, std::true_type{});
    } else {
#pragma unroll
      for (int jj = 0; jj < VW; ++jj)
        if (wave + kShWaves * jj < nv) blend_view(jj, std::false_type{});
    }
  }
  if (x < a.nx) {
    float4* out = static_cast<float4*>(a.out);
#pragma unroll
    for (int jj = 0; jj < VW; ++jj) {
      const int j = wave + kShWaves * jj;
      if (j < nv) out[((size_t)a.perm[v0 + j] * a.ny + y) * a.nx + x] = make_float4(Qr[jj], Qg[jj], Qb[jj], Tr[jj]);
    }
  }
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
hipError_t launch_composite(CompositeArgs& a, const ShView& sv, hipStream_t s) {
  // the row kernel unless LF_COMPOSITE_KERNEL=general asks for the per-pixel one (tests)
  const char* kern = getenv("LF_COMPOSITE_KERNEL");
  if (!(kern && std::strcmp(kern, "general") == 0)) {
    view_groups(a, kShGroup);
    const int nseg = (a.nx + kShSeg - 1) / kShSeg;
    const int total = a.n_groups * nseg * a.ny;
    const dim3 grid((unsigned)(((total + 7) / 8) * 8)), block(kShSeg * kShWaves);
    const size_t lds = (size_t)(kShWinBytes / (sh_texel_floats(NC) * 4)) * sh_texel_floats(NC) * 4;
    if (a.interp == LF_BILINEAR)
      hipLaunchKernelGGL((composite_sh_rows<NC, true>), grid, block, lds, s, a, sv, nseg, total);
    else
      hipLaunchKernelGGL((composite_sh_rows<NC, false>), grid, block, lds, s, a, sv, nseg, total);
    return hipGetLastError();
  }
  const int64_t n = (int64_t)a.n_views * a.ny * a.nx;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (a.interp == LF_BILINEAR) hipLaunchKernelGGL((composite_sh<NC, true>), grid, dim3(256), 0, s, a, sv);
  else hipLaunchKernelGGL((composite_sh<NC, false>), grid, dim3(256), 0, s, a, sv);
  return hipGetLastError();
}

}  // namespace

hipError_t composite_sh_launch(CompositeArgs& a, int n_coef, const ShView& sv, hipStream_t s) {
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
