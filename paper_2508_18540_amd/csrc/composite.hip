// Swizzle blending of the sweeping planes into light-field views (Sec. 4.3, Eqs. 6-7,
// Alg. 1 steps 6-11) for gfx950.
//
// Texel coordinates follow Eq. 6 in affine form.  For plane k at base depth d:
//   z = d - D_fwd, q = d / z, w = (1 - d / D_focal) / z,
//   bx = (f'_x / f_x) q,  gx = f'_x w,  Cx[v] = c'_x + gx dx_v  (+1/2 for nearest),
//   X = bx (x - c_x) + Cx[v],
// every operation a correctly rounded float32 operation (the library is compiled with
// -ffp-contract=off and fuses only where fmaf is written).  Nearest sampling takes the
// texel floor(X); bilinear takes floor(X), floor(X)+1 with weight X - floor(X).
//
// Row kernel (all views share dy, e.g. a horizontal-parallax quilt).  Y depends only on
// (k, y), so one work-group owns one output row y for a group of G views and every x of
// a row segment.  Per plane it stages the plane row Y_k(y) (bilinear: the two rows,
// pre-blended vertically) into LDS as float32 with transparent guard texels on both
// sides, so each sample is one clamped LDS read plus four FMAs into float32 registers
// that hold (Q, T) for G views.  Planes whose row misses the plane are skipped.
// General kernel (views with different dy): one thread per output pixel, texels read
// straight from global memory.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kRowThreads = 512;
constexpr int kRowLdsBytes = 60 * 1024;

struct PlaneCo {
  float bx, by, gx, gy;
};

__device__ __forceinline__ PlaneCo plane_co(float d, const Consts& c) {
  const float z = d - c.d_fwd;
  const float q = d / z;
  const float w = (1.0f - d * c.inv_focal) / z;
  return {c.ratio_x * q, c.ratio_y * q, c.fpx * w, c.fpy * w};
}

template <typename T>
__device__ __forceinline__ float4 load_texel(const T* p, size_t i);

template <>
__device__ __forceinline__ float4 load_texel<float>(const float* p, size_t i) {
  return reinterpret_cast<const float4*>(p)[i];
}

template <>
__device__ __forceinline__ float4 load_texel<__half>(const __half* p, size_t i) {
  const uint2 u = reinterpret_cast<const uint2*>(p)[i];
  const __half2 lo = *reinterpret_cast<const __half2*>(&u.x);
  const __half2 hi = *reinterpret_cast<const __half2*>(&u.y);
  const float2 a = __half22float2(lo), b = __half22float2(hi);
  return make_float4(a.x, a.y, b.x, b.y);
}

template <>
__device__ __forceinline__ float4 load_texel<__hip_bfloat16>(const __hip_bfloat16* p, size_t i) {
  const uint2 u = reinterpret_cast<const uint2*>(p)[i];
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                     __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
}

template <typename T>
__device__ __forceinline__ void store_pixel(T* out, size_t i, float r, float g, float b, float t);

template <>
__device__ __forceinline__ void store_pixel<float>(float* out, size_t i, float r, float g, float b, float t) {
  reinterpret_cast<float4*>(out)[i] = make_float4(r, g, b, t);
}

template <>
__device__ __forceinline__ void store_pixel<__half>(__half* out, size_t i, float r, float g, float b, float t) {
  const __half2 lo = __floats2half2_rn(r, g);
  const __half2 hi = __floats2half2_rn(b, t);
  uint2 u;
  u.x = *reinterpret_cast<const uint32_t*>(&lo);
  u.y = *reinterpret_cast<const uint32_t*>(&hi);
  reinterpret_cast<uint2*>(out)[i] = u;
}

__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float w) {
  return make_float4(fmaf(w, b.x - a.x, a.x), fmaf(w, b.y - a.y, a.y), fmaf(w, b.z - a.z, a.z),
                     fmaf(w, b.w - a.w, a.w));
}

// ---------------------------------------------------------------------------------------
// Row kernel.  grid = (ny, view groups, x segments), block = kRowThreads (or fewer).
// LDS: nearest  -> row[i] = texel i-1, i in [0, wp+2)   (texels -1 and wp are zero)
//      bilinear -> row[e] = (t_{e-2}, t_{e-1} - t_{e-2}), e in [0, wp+3)
// ---------------------------------------------------------------------------------------
template <typename PT, typename OT, int G, bool BIL>
__global__ __launch_bounds__(kRowThreads) void composite_rows(CompositeArgs a, int seg_len) {
  extern __shared__ float4 lds[];
  __shared__ float sC[G];
  const int y = blockIdx.x;
  const int v0 = blockIdx.y * G;
  const int nv = min(G, a.n_views - v0);
  const int tid = threadIdx.x;
  const int x = blockIdx.z * seg_len + tid;
  const int wp = a.wp, hp = a.hp;
  const PT* planes = static_cast<const PT*>(a.planes);
  const float xr = (float)x - a.c.cx;
  const float yr = (float)y - a.c.cy;
  const float dy0 = a.dy[0];

  float Qr[G], Qg[G], Qb[G], Tr[G];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    Qr[j] = Qg[j] = Qb[j] = 0.0f;
    Tr[j] = 1.0f;
  }

  for (int k = 0; k < a.K; ++k) {
    const float d = a.depth[k];
    const PlaneCo pc = plane_co(d, a.c);
    const float cy = a.c.cpy + pc.gy * dy0;
    int iy0;
    float wy = 0.0f;
    if (!BIL) {
      const float Y = pc.by * yr + (cy + 0.5f);
      iy0 = __float2int_rd(Y);
      if (!(iy0 >= 0 && iy0 < hp)) continue;           // uniform across the work-group
    } else {
      const float Y = pc.by * yr + cy;
      const float fy0 = floorf(Y);
      wy = Y - fy0;
      iy0 = __float2int_rd(fy0);
      if (!(iy0 >= -1 && iy0 < hp)) continue;
    }
    __syncthreads();                                     // previous plane's samples are done
    const size_t plane_base = (size_t)k * hp * wp;
    if (!BIL) {
      const size_t rbase = plane_base + (size_t)iy0 * wp;
      for (int i = tid; i < wp + 2; i += blockDim.x) {
        const int ix = i - 1;
        lds[i] = (ix >= 0 && ix < wp) ? load_texel(planes, rbase + ix) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    } else {
      const bool r0 = iy0 >= 0, r1 = iy0 + 1 < hp;
      const size_t b0 = plane_base + (size_t)iy0 * wp, b1 = b0 + wp;
      for (int e = tid; e < wp + 3; e += blockDim.x) {
        const int ix = e - 2;
        float4 t0 = make_float4(0.f, 0.f, 0.f, 0.f), t1 = t0;
        if (ix >= 0 && ix < wp) {
          const float4 u = r0 ? load_texel(planes, b0 + ix) : t0;
          const float4 w = r1 ? load_texel(planes, b1 + ix) : t0;
          t0 = lerp4(u, w, wy);
        }
        if (ix + 1 >= 0 && ix + 1 < wp) {
          const float4 u = r0 ? load_texel(planes, b0 + ix + 1) : t1;
          const float4 w = r1 ? load_texel(planes, b1 + ix + 1) : t1;
          t1 = lerp4(u, w, wy);
        }
        lds[2 * e] = t0;
        lds[2 * e + 1] = make_float4(t1.x - t0.x, t1.y - t0.y, t1.z - t0.z, t1.w - t0.w);
      }
    }
    if (tid < nv) {
      const float cx = a.c.cpx + pc.gx * a.dx[v0 + tid];
      sC[tid] = BIL ? cx : cx + 0.5f;
    }
    __syncthreads();
    const float bxr = pc.bx * xr;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      if (j < nv) {
        const float X = bxr + sC[j];
        float4 s;
        if (!BIL) {
          const int ix = min(max(__float2int_rd(X), -1), wp);
          s = lds[ix + 1];
        } else {
          const float fx0 = floorf(X);
          const float w = X - fx0;
          const int ix = min(max(__float2int_rd(fx0), -2), wp);
          const float4 t = lds[2 * (ix + 2)];
          const float4 dd = lds[2 * (ix + 2) + 1];
          s = make_float4(fmaf(w, dd.x, t.x), fmaf(w, dd.y, t.y), fmaf(w, dd.z, t.z), fmaf(w, dd.w, t.w));
        }
        Qr[j] = fmaf(Tr[j], s.x, Qr[j]);
        Qg[j] = fmaf(Tr[j], s.y, Qg[j]);
        Qb[j] = fmaf(Tr[j], s.z, Qb[j]);
        Tr[j] = fmaf(-Tr[j], s.w, Tr[j]);
      }
    }
  }
  if (tid < seg_len && x < a.nx) {
    OT* out = static_cast<OT*>(a.out);
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (j < nv) store_pixel(out, ((size_t)(v0 + j) * a.ny + y) * a.nx + x, Qr[j], Qg[j], Qb[j], Tr[j]);
  }
}

// ---------------------------------------------------------------------------------------
// General kernel: any per-view (dx, dy).  One thread per output pixel.
// ---------------------------------------------------------------------------------------
template <typename PT, typename OT, bool BIL>
__global__ __launch_bounds__(256) void composite_general(CompositeArgs a) {
  const int64_t n = (int64_t)a.n_views * a.ny * a.nx;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % a.nx);
  const int y = (int)((i / a.nx) % a.ny);
  const int v = (int)(i / ((int64_t)a.nx * a.ny));
  const PT* planes = static_cast<const PT*>(a.planes);
  const float xr = (float)x - a.c.cx, yr = (float)y - a.c.cy;
  const float dx = a.dx[v], dy = a.dy[v];
  float Qr = 0.f, Qg = 0.f, Qb = 0.f, Tr = 1.f;
  for (int k = 0; k < a.K; ++k) {
    const PlaneCo pc = plane_co(a.depth[k], a.c);
    const float cx = a.c.cpx + pc.gx * dx;
    const float cy = a.c.cpy + pc.gy * dy;
    const size_t base = (size_t)k * a.hp * a.wp;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!BIL) {
      const float X = pc.bx * xr + (cx + 0.5f);
      const float Y = pc.by * yr + (cy + 0.5f);
      const int ix = __float2int_rd(X), iy = __float2int_rd(Y);
      if (ix >= 0 && ix < a.wp && iy >= 0 && iy < a.hp) s = load_texel(planes, base + (size_t)iy * a.wp + ix);
    } else {
      const float X = pc.bx * xr + cx;
      const float Y = pc.by * yr + cy;
      const float fx0 = floorf(X), fy0 = floorf(Y);
      const float wx = X - fx0, wy = Y - fy0;
      const int ix = __float2int_rd(fx0), iy = __float2int_rd(fy0);
      float4 t[2][2];
#pragma unroll
      for (int oy = 0; oy < 2; ++oy)
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
          const int xx = ix + ox, yy = iy + oy;
          t[oy][ox] = (xx >= 0 && xx < a.wp && yy >= 0 && yy < a.hp)
                          ? load_texel(planes, base + (size_t)yy * a.wp + xx)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      s = lerp4(lerp4(t[0][0], t[0][1], wx), lerp4(t[1][0], t[1][1], wx), wy);
    }
    Qr = fmaf(Tr, s.x, Qr);
    Qg = fmaf(Tr, s.y, Qg);
    Qb = fmaf(Tr, s.z, Qb);
    Tr = fmaf(-Tr, s.w, Tr);
  }
  store_pixel(static_cast<OT*>(a.out), (size_t)i, Qr, Qg, Qb, Tr);
}

__global__ void plane_coeffs_kernel(CompositeArgs a, float* bx, float* by, float* cx, float* cy,
                                    float* cxn, float* cyn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.K * a.n_views) return;
  const int k = i / a.n_views, v = i % a.n_views;
  const PlaneCo pc = plane_co(a.depth[k], a.c);
  const float X = a.c.cpx + pc.gx * a.dx[v];
  const float Y = a.c.cpy + pc.gy * a.dy[v];
  if (v == 0) {
    bx[k] = pc.bx;
    by[k] = pc.by;
  }
  cx[i] = X;
  cy[i] = Y;
  cxn[i] = X + 0.5f;
  cyn[i] = Y + 0.5f;
}

template <int G>
int pick_cost(int V) { return ((V + G - 1) / G) * (G + 4); }

template <typename PT, typename OT, bool BIL>
hipError_t launch_rows(const CompositeArgs& a, int G, hipStream_t s) {
  const int nseg = (a.nx + kRowThreads - 1) / kRowThreads;
  const int seg = (a.nx + nseg - 1) / nseg;
  const int threads = ((seg + 63) / 64) * 64;
  const size_t lds = BIL ? (size_t)(a.wp + 3) * 32 : (size_t)(a.wp + 2) * 16;
  const dim3 grid(a.ny, (a.n_views + G - 1) / G, nseg);
  switch (G) {
    case 4: hipLaunchKernelGGL((composite_rows<PT, OT, 4, BIL>), grid, dim3(threads), lds, s, a, seg); break;
    case 8: hipLaunchKernelGGL((composite_rows<PT, OT, 8, BIL>), grid, dim3(threads), lds, s, a, seg); break;
    case 12: hipLaunchKernelGGL((composite_rows<PT, OT, 12, BIL>), grid, dim3(threads), lds, s, a, seg); break;
    default: hipLaunchKernelGGL((composite_rows<PT, OT, 16, BIL>), grid, dim3(threads), lds, s, a, seg); break;
  }
  return hipGetLastError();
}

template <typename PT, typename OT>
hipError_t dispatch_interp(const CompositeArgs& a, bool rows, int G, hipStream_t s) {
  if (rows)
    return a.interp == LF_BILINEAR ? launch_rows<PT, OT, true>(a, G, s) : launch_rows<PT, OT, false>(a, G, s);
  const int64_t n = (int64_t)a.n_views * a.ny * a.nx;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (a.interp == LF_BILINEAR)
    hipLaunchKernelGGL((composite_general<PT, OT, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((composite_general<PT, OT, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename PT>
hipError_t dispatch_out(const CompositeArgs& a, bool rows, int G, hipStream_t s) {
  return a.out_dtype == LF_F16 ? dispatch_interp<PT, __half>(a, rows, G, s)
                               : dispatch_interp<PT, float>(a, rows, G, s);
}

}  // namespace

hipError_t composite_launch(const CompositeArgs& a, hipStream_t s) {
  bool same_dy = true;
  for (int v = 1; v < a.n_views; ++v) same_dy = same_dy && a.dy[v] == a.dy[0];
  const size_t lds = a.interp == LF_BILINEAR ? (size_t)(a.wp + 3) * 32 : (size_t)(a.wp + 2) * 16;
  const bool rows = same_dy && lds <= (size_t)kRowLdsBytes;
  int G = 16, best = pick_cost<16>(a.n_views);
  if (pick_cost<12>(a.n_views) < best) { G = 12; best = pick_cost<12>(a.n_views); }
  if (pick_cost<8>(a.n_views) < best) { G = 8; best = pick_cost<8>(a.n_views); }
  if (pick_cost<4>(a.n_views) < best) { G = 4; best = pick_cost<4>(a.n_views); }
  switch (a.plane_dtype) {
    case LF_F16: return dispatch_out<__half>(a, rows, G, s);
    case LF_BF16: return dispatch_out<__hip_bfloat16>(a, rows, G, s);
    default: return dispatch_out<float>(a, rows, G, s);
  }
}

hipError_t plane_coeffs_launch(const CompositeArgs& a, float* bx, float* by, float* cx, float* cy,
                               float* cxn, float* cyn, hipStream_t s) {
  const int n = a.K * a.n_views;
  hipLaunchKernelGGL(plane_coeffs_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, bx, by, cx, cy, cxn, cyn);
  return hipGetLastError();
}

}  // namespace lf
