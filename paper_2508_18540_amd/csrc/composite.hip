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
// A small table kernel evaluates these coefficients once per launch: per (view group, plane)
// (bx, by, the row offset Cy of the group's dy, a validity flag) and per (plane, view) Cx.
//
// Row kernel.  Views are grouped by their vertical offset dy: a horizontal-parallax quilt is
// one class, a Vx x Vy quilt Vy classes, an arbitrary view list as many classes as distinct
// dy.  Within a class Y depends only on (k, y), so one work-group owns one output row y for a
// group of up to G views of one class and every x of a row segment; (Q, T) of the group's
// views live in float32 registers.  Per plane it stages
// into LDS the window of the plane row Y_k(y) (bilinear: the two rows blended
// vertically) that holds every sample of the work-group, double-buffered so the next
// plane's texels are in flight while the current one is sampled.  A sample is then one
// LDS read plus four FMAs; the per-view offsets come through scalar loads.  Planes whose
// row misses the plane are skipped.
// General kernel (planes too wide for the row kernel's window buffer): one thread per output
// pixel, texels read straight from global memory.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "lf_internal.h"
#include "lds_sync.h"

namespace lf {
namespace {

constexpr int kRowThreads = 256;

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

template <>
__device__ __forceinline__ float4 load_texel<uint8_t>(const uint8_t* p, size_t i) {
  // UNORM8: code / 255 (to float32 rounding)
  const uint32_t u = reinterpret_cast<const uint32_t*>(p)[i];
  constexpr float s = 1.0f / 255.0f;
  return make_float4((float)(u & 0xffu) * s, (float)((u >> 8) & 0xffu) * s, (float)((u >> 16) & 0xffu) * s,
                     (float)(u >> 24) * s);
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

// a if ok, else zero, selected per component (a select of whole vectors can turn into a
// select of their addresses, which forces them into scratch memory)
__device__ __forceinline__ float4 keep_if(bool ok, float4 a) {
  return make_float4(ok ? a.x : 0.0f, ok ? a.y : 0.0f, ok ? a.z : 0.0f, ok ? a.w : 0.0f);
}

__device__ __forceinline__ uint2 keep_if(bool ok, uint2 a) { return make_uint2(ok ? a.x : 0u, ok ? a.y : 0u); }

__device__ __forceinline__ uint32_t keep_if(bool ok, uint32_t a) { return ok ? a : 0u; }

// Four UNORM8 codes as four FP16 numbers 0..255 (exact).
__device__ __forceinline__ uint2 codes_to_half4(uint32_t u) {
  const __half2 lo = __floats2half2_rn((float)(u & 0xffu), (float)((u >> 8) & 0xffu));
  const __half2 hi = __floats2half2_rn((float)((u >> 16) & 0xffu), (float)(u >> 24));
  return make_uint2(*reinterpret_cast<const uint32_t*>(&lo), *reinterpret_cast<const uint32_t*>(&hi));
}

__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float w) {
  return make_float4(fmaf(w, b.x - a.x, a.x), fmaf(w, b.y - a.y, a.y), fmaf(w, b.z - a.z, a.z),
                     fmaf(w, b.w - a.w, a.w));
}

// ---------------------------------------------------------------------------------------
// Table kernel: pt[g][k] = (bx, by, Cy, L) for view group g's dy (L: 0 for an invalid plane,
// else the lane count of the backward's accumulation phases), ct[k][p] = Cx of the
// view at position p of the grouped order, rows padded by kViewPad positions (the padding
// repeats the last position) so a group's G offsets can always be read, and pm[g][k] = the
// least and greatest Cx of group g's view slots (its views, and with `slots` the positions
// after a short group's end up to `slots` in all: kernels that sample every slot read them).
// Nearest sampling folds the 1/2 of floor(X + 1/2) into Cx and Cy.
// ---------------------------------------------------------------------------------------
constexpr int kViewPad = 24;                  // >= the largest view group - 1

__host__ __device__ inline int ct_stride(int V) { return V + kViewPad; }

__device__ __forceinline__ float view_cx(const CompositeArgs& a, const PlaneCo& pc, int p) {
  const float cx = a.c.cpx + pc.gx * a.dx[a.perm[min(p, a.n_views - 1)]];
  return a.interp == LF_BILINEAR ? cx : cx + 0.5f;
}

__global__ void coeff_table(CompositeArgs a, float4* __restrict__ pt, float* __restrict__ ct, float2* __restrict__ pm,
                            int slots) {
  const int S = ct_stride(a.n_views);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && a.spill) *a.spill = 0u;
  if (i >= a.K * S) return;
  const int k = i / S, p = i % S;
  const int v = a.perm[min(p, a.n_views - 1)];
  const float d = a.depth[k];
  const PlaneCo pc = plane_co(d, a.c);
  const float half = a.interp == LF_BILINEAR ? 0.0f : 0.5f;
  const float cx = a.c.cpx + pc.gx * a.dx[v];
  ct[i] = a.interp == LF_BILINEAR ? cx : cx + half;
  if (p < a.n_groups) {
    const int q0 = a.vgroup[p] & 0xffu, nq = a.vgroup[p] >> 8;
    const float cy = a.c.cpy + pc.gy * a.dy[a.perm[q0]];
    // w: 0 for a plane at or behind the reference camera, else the lane count L the
    // backward's updates need: lanes L apart never share a texel floor(X) when their
    // coordinates differ by at least 1.  They differ by L bx up to the two roundings of each
    // X, under 4e-3 in all for |X|, |bx xr| < 2^14, so L bx must exceed 1 by 1e-2.
    const float L = pc.bx > 0.0f ? fminf(floorf(1.01f / pc.bx) + 1.0f, 64.0f) : 64.0f;
    pt[(size_t)p * a.K + k] = make_float4(pc.bx, pc.by, a.interp == LF_BILINEAR ? cy : cy + half,
                                          d - a.c.d_fwd > 0.0f ? L : 0.0f);
    // least and greatest Cx over the group's positions, padded to `slots` (a kernel that
    // samples a fixed number of views reads the positions after a short group's end)
    const int qe = min(q0 + max(nq, slots), S);
    float cmin = view_cx(a, pc, q0), cmax = cmin;
    for (int q = q0 + 1; q < qe; ++q) {
      const float c = view_cx(a, pc, q);
      cmin = fminf(cmin, c);
      cmax = fmaxf(cmax, c);
    }
    pm[(size_t)p * a.K + k] = make_float2(cmin, cmax);
  }
}

// ---------------------------------------------------------------------------------------
// Row kernel.  One work-group per (view group, x segment, output row), block = up to
// kRowThreads threads, one output pixel x per thread and up to G views (one group) per
// work-group.  The groups and segments of a row stage the same plane rows, so the logical
// tiles (group fastest, then segment, then row) are dealt to the 8 XCDs in contiguous runs
// (work-group w runs on XCD w mod 8): the work-groups that share plane rows run at about
// the same time and meet in one L2.
//
// Planes are processed in batches of kBatch.  A prologue (one thread per plane) derives
// the plane row and the texel window [f0, f0 + len) that contains every sample of this
// work-group: X is monotone in x and in Cx, so its extremes are the samples at the segment
// ends with the extreme offsets.  Windows are staged into LDS with zeros outside the
// plane, and a sample is floor(X) - f0 without a clamp.
// The row kernel takes the 64-pixel segments the one-wave kernel (below) leaves: those with
// a window longer than that kernel's buffer.  A window longer than its own buffer (kWin)
// falls back to the whole row [-2, wp + 1], with samples clamped onto its zero guards.
//   nearest  : win[i] = texel f0 + i (FP16 planes keep FP16 texels, others float32)
//   bilinear : win[2i] = t(f0 + i), win[2i+1] = t(f0 + i + 1) - t(f0 + i), float32, with t
//              the row pair blended vertically by the plane's weight wy
// ---------------------------------------------------------------------------------------
constexpr int kBatch = 64;
constexpr int kWin = 2048;                    // float4 entries per window buffer
constexpr int kWinStride = kWin + 2;          // plus a trash slot for inactive stores
constexpr int kPrefetch = kWin / kRowThreads; // window entries prefetched per thread (nearest)
constexpr int kWaveWin = 256;                 // window entries of the one-wave kernel's buffers

// Table pointers in the global address space: a kernel that reads them from device memory
// (the batch's jobs) then still loads through them with global, not flat, instructions.
typedef const float4 __attribute__((address_space(1)))* GF4;
typedef const float __attribute__((address_space(1)))* GF1;
typedef const float2 __attribute__((address_space(1)))* GF2;
// wave-uniform table reads through the constant address space: scalar loads into SGPRs
typedef const float __attribute__((address_space(4)))* CF1;
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 ld4(GF4 p) {
  const v4f v = *(const v4f __attribute__((address_space(1)))*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ld2(GF2 p) {
  const v2f v = *(const v2f __attribute__((address_space(1)))*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float4 ld4(const float4* p) { return *p; }
__device__ __forceinline__ float2 ld2(const float2* p) { return *p; }

// Whether every plane that view group `pt`/`pm` (the group's table rows) samples has, for
// the 64 pixels [xs0, xs0 + 64) of row y, a window of at most kWaveWin entries (the
// one-wave kernel's); wave uniform.  A plane is sampled unless it is invalid, its row lies
// outside the plane, or its window lies wholly outside the row (transparent texels only).
// The one-wave kernel and the row kernel decide each segment with this same function.
template <bool BIL, typename P4, typename P2>
__device__ bool wave_fits(const CompositeArgs& a, P4 pt, P2 pm, int xs0, int y) {
  const int lane = threadIdx.x & 63;
  const float yr = (float)y - a.c.cy;
  const float xr_lo = (float)xs0 - a.c.cx, xr_hi = (float)(xs0 + 63) - a.c.cx;
  const int cap = BIL ? kWaveWin / 2 : kWaveWin;
  bool slow = false;
  for (int kb = 0; kb < a.K; kb += 64) {
    const int k = kb + lane;
    bool s = false;
    if (k < a.K) {
      const float4 p = ld4(pt + k);
      const float2 cr = ld2(pm + k);
      const float Y = p.y * yr + p.z;
      const int iy = (int)floorf(Y);
      const bool ok = p.w != 0.0f && iy >= (BIL ? -1 : 0) && iy < a.hp;
      const float lo = floorf(p.x * xr_lo + cr.x);
      const float hi = floorf(p.x * xr_hi + cr.y) + (BIL ? 1.0f : 0.0f);
      const bool outside = hi < 0.0f || lo > (float)(a.wp - 1);
      s = ok && !outside && !(hi - lo + 1.0f <= (float)cap);
    }
    slow = slow || __builtin_amdgcn_ballot_w64(s) != 0;
  }
  return !slow;
}
constexpr int kSub = 4;                       // views sampled per scheduling block

struct PlaneInfo {
  float wy;
  int32_t iy, f0, len;
};

__device__ __forceinline__ int cvt_flr(float x) {
  int r;
  asm volatile("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// LDS texel of the nearest window: FP16 planes stay FP16 (8 bytes), UNORM8 planes become
// their codes as FP16 (exact: 0..255; the blend scales by 1/255), others are float32.  FP16
// texels let the blend use mixed-precision FMAs (no conversion instructions).
template <typename PT> struct LdsTexel { using type = float4; };
template <> struct LdsTexel<__half> { using type = uint2; };
template <> struct LdsTexel<uint8_t> { using type = uint2; };

template <typename LT>
__device__ __forceinline__ float4 lds_texel(const char* p);

template <>
__device__ __forceinline__ float4 lds_texel<float4>(const char* p) {
  return *reinterpret_cast<const float4*>(p);
}

template <>
__device__ __forceinline__ float4 lds_texel<uint2>(const char* p) {
  const uint2 u = *reinterpret_cast<const uint2*>(p);
  const __half2 lo = *reinterpret_cast<const __half2*>(&u.x);
  const __half2 hi = *reinterpret_cast<const __half2*>(&u.y);
  return make_float4(__low2float(lo), __high2float(lo), __low2float(hi), __high2float(hi));
}

// Bilinear window entry i of a plane: the vertically blended texel and its forward difference.
template <typename PT>
__device__ __forceinline__ void bilinear_entry(const PT* __restrict__ planes, size_t pbase, int wp, int hp,
                                               const PlaneInfo& pi, int i, float4& t0, float4& dd) {
  const int ix = pi.f0 + i;
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  const bool r0 = pi.iy >= 0, r1 = pi.iy + 1 < hp;
  const size_t b0 = pbase + (size_t)pi.iy * wp, b1 = b0 + wp;
  float4 t1 = z;
  t0 = z;
  if (ix >= 0 && ix < wp) t0 = lerp4(r0 ? load_texel(planes, b0 + ix) : z, r1 ? load_texel(planes, b1 + ix) : z, pi.wy);
  if (ix + 1 >= 0 && ix + 1 < wp)
    t1 = lerp4(r0 ? load_texel(planes, b0 + ix + 1) : z, r1 ? load_texel(planes, b1 + ix + 1) : z, pi.wy);
  dd = make_float4(t1.x - t0.x, t1.y - t0.y, t1.z - t0.z, t1.w - t0.w);
}

template <typename PT, typename OT, int G, bool BIL>
__global__ __launch_bounds__(kRowThreads) void composite_rows(CompositeArgs a, int seg_len,
                                                              int nseg, int total,
                                                              const float4* __restrict__ pt,
                                                              const float* __restrict__ ct,
                                                              const float2* __restrict__ pm) {
  using LT = typename std::conditional<BIL, float4, typename LdsTexel<PT>::type>::type;
  constexpr bool RAW = !std::is_same<LT, float4>::value;   // FP16 texels in LDS (FP16 / UNORM8 planes)
  constexpr bool U8 = RAW && std::is_same<PT, uint8_t>::value;   // samples are codes: scale by 1/255
  using RT = typename std::conditional<U8, uint32_t, uint2>::type;   // raw texel as fetched
  // nearest FP32 / FP16 / UNORM8 windows are fetched with buffer loads over the plane row:
  // the hardware's range check returns zero outside the row, so no clamp or mask is needed
  constexpr bool BUF = !BIL && (RAW || std::is_same<PT, float>::value);
  constexpr int kTexelBytes = RAW ? (int)sizeof(RT) : 16;
  constexpr int W = kWin, WS = kWinStride;
  constexpr int PF = (W / kRowThreads) / (BIL ? 2 : 1);    // window entries each thread fetches
  extern __shared__ float4 win[];                          // 2 buffers of W float4
  __shared__ PlaneInfo pinfo[kBatch];
  __shared__ int slist[kBatch];
  __shared__ int scount;                                   // valid planes of the batch
  const int wg = blockIdx.x;
  const int per = (total + 7) / 8;
  const int lg = (wg % 8) * per + wg / 8;
  if (lg >= total) return;                                 // whole work-group: grid padded to 8 per
  // the one-wave kernel ran before (64-pixel tiles) and took every segment: nothing to do
  if (a.tile != 256 && a.spill && *a.spill == 0u) return;
  const int gi = lg % a.n_groups, rest = lg / a.n_groups;
  const int y = rest / nseg;
  const uint32_t gd = a.vgroup[gi];
  const int v0 = gd & 0xffu;                               // group's first position in perm
  const int nv = gd >> 8;
  pt += (size_t)gi * a.K;
  pm += (size_t)gi * a.K;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int xs0 = (rest % nseg) * seg_len;
  const int x = xs0 + tid;
  const int xs1 = min(xs0 + seg_len, a.nx) - 1;
  const int wp = a.wp, hp = a.hp, V = ct_stride(a.n_views);
  const PT* __restrict__ planes = static_cast<const PT*>(a.planes);
  const float xr = (float)x - a.c.cx;
  const float yr = (float)y - a.c.cy;
  const float xr_lo = (float)xs0 - a.c.cx, xr_hi = (float)xs1 - a.c.cx;
  const size_t plane_elems = (size_t)hp * wp;

  // the window of plane k for this work-group: row iy (bilinear: first of two, weight wy),
  // [lo, hi] as floats, and whether the plane is sampled at all (ok)
  auto window = [&](int k, float& lo, float& hi, int& iy, float& wy) {
    const float4 p = pt[k];                                // (bx, by, Cy, valid)
    wy = 0.0f;
    bool ok = p.w != 0.0f;
    if (!BIL) {
      iy = __float2int_rd(p.y * yr + p.z);
      ok = ok && iy >= 0 && iy < hp;
    } else {
      const float Y = p.y * yr + p.z;
      const float fy0 = floorf(Y);
      wy = Y - fy0;
      iy = __float2int_rd(fy0);
      ok = ok && iy >= -1 && iy < hp;
    }
    // the least and greatest Cx over the group's G slots (the table's padded extents: the
    // slots past a short group's end are sampled too, their results dropped)
    const float2 cr = pm[k];
    lo = floorf(p.x * xr_lo + cr.x);
    hi = floorf(p.x * xr_hi + cr.y) + (BIL ? 1.0f : 0.0f);
    return ok;
  };
  // a window fits a buffer of `cap` entries (and the fetch of PF entries per thread)
  auto fits = [&](float lo, float hi, int cap) { return lo >= -1.0e9f && hi <= 1.0e9f && hi - lo + 1.0f <= (float)cap; };
  // this wave's 64-pixel segment is the one-wave kernel's when its windows fit that
  // kernel's buffer (segments start at multiples of 64: seg_len is) and 64-pixel tiles are
  // in use; the work-group returns when all its waves' are
  const int wx0 = xs0 + (tid & ~63);
  const bool wave_done = wx0 >= a.nx || (a.tile != 256 && wave_fits<BIL>(a, pt, pm, wx0, y));
  if (__syncthreads_and(wave_done)) return;
  float Qr[G], Qg[G], Qb[G], Tr[G];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    Qr[j] = Qg[j] = Qb[j] = 0.0f;
    Tr[j] = 1.0f;
  }

  for (int kb = 0; kb < a.K; kb += kBatch) {
    const int nk = min(kBatch, a.K - kb);
    __syncthreads();                                       // previous batch fully consumed
    if (tid == 0) scount = 0;
    __syncthreads();
    if (tid < nk) {
      const int k = kb + tid;
      PlaneInfo pi;
      float lo, hi;
      bool ok = window(k, lo, hi, pi.iy, pi.wy);
      // a window must fit the buffer and be covered by the fetch (PF entries per thread)
      const int cap = min(BIL ? W / 2 : W, PF * nt);
      if (fits(lo, hi, cap)) {
        pi.f0 = (int)lo;
        pi.len = (int)(hi - lo) + 1;
        // a window wholly outside the row samples only transparent texels, which leave
        // (Q, T) unchanged exactly; skipping it also keeps every fetched column within
        // (-cap, wp + cap), where a buffer offset cannot wrap
        if (!BIL) ok = ok && hi >= 0.0f && lo <= (float)(wp - 1);
      } else {
        pi.f0 = -2;                                        // whole row [-2, wp + 1], clamped
        pi.len = wp + 4;
      }
      pinfo[tid] = pi;
      if (ok) slist[atomicAdd(&scount, 1)] = tid;          // order restored below
    }
    __syncthreads();
    const int nvalid = __builtin_amdgcn_readfirstlane(scount);
    if (nvalid == 0) continue;
    if (tid == 0) {                                        // front-to-back order of the valid planes
      for (int i = 1; i < nvalid; ++i) {
        const int v = slist[i];
        int j = i - 1;
        while (j >= 0 && slist[j] > v) {
          slist[j + 1] = slist[j];
          --j;
        }
        slist[j + 1] = v;
      }
    }
    __syncthreads();

    // Window fetch, split in two: fetch() issues every load of the next plane's window with
    // no branches, so the loads stay in flight while the current plane is sampled; store()
    // writes them to LDS.  Nearest FP32 / FP16 / UNORM8 rows use buffer loads, which return
    // zero outside the row; the other forms clamp their addresses (always valid) and store()
    // masks the out-of-plane texels to zero.
    float4 ra[RAW ? 1 : PF], rb[BIL ? PF : 1], rc[BIL ? PF : 1], rd[BIL ? PF : 1];
    RT praw[RAW ? PF : 1];
    uint32_t valid = 0;                                    // bit (q * 4 + r): raw texel in the plane
    auto fetch = [&](int k) {
      const PlaneInfo pi = pinfo[k];
      const size_t pbase = (size_t)(kb + k) * plane_elems;
      valid = 0;
      // (the row of a fetched plane lies in the plane: planes with iy outside it are not valid)
      const char* rowp = reinterpret_cast<const char*>(planes) + (BUF ? (pbase + (size_t)pi.iy * wp) * kTexelBytes : 0);
      const auto rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(rowp), (short)0, wp * kTexelBytes, 0x00020000);
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        if (q * nt >= pi.len) break;                       // uniform: the window is shorter
        const int i = tid + q * nt;
        const int ix = pi.f0 + i;
        const bool in = i < pi.len;
        if constexpr (BUF) {
          (void)in;
          const uint32_t off = (uint32_t)ix * (uint32_t)kTexelBytes;   // ix < 0 wraps past the row
          if constexpr (U8) praw[q] = (RT)__builtin_amdgcn_raw_buffer_load_b32(rsrc, off, 0, 0);
          else if constexpr (RAW) praw[q] = __builtin_bit_cast(RT, __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, 0, 0));
          else ra[q] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0));
        } else if constexpr (!BIL) {
          const bool ok = in && ix >= 0 && ix < wp;
          const size_t at = pbase + (size_t)pi.iy * wp + (size_t)min(max(ix, 0), wp - 1);
          if constexpr (RAW) praw[q] = reinterpret_cast<const RT*>(planes)[at];
          else ra[q] = load_texel(planes, at);
          valid |= (ok ? 1u : 0u) << (q * 4);
        } else {
          const int r0 = min(max(pi.iy, 0), hp - 1), r1 = min(max(pi.iy + 1, 0), hp - 1);
          const size_t c0 = (size_t)min(max(ix, 0), wp - 1), c1 = (size_t)min(max(ix + 1, 0), wp - 1);
          ra[q] = load_texel(planes, pbase + (size_t)r0 * wp + c0);
          rb[q] = load_texel(planes, pbase + (size_t)r1 * wp + c0);
          rc[q] = load_texel(planes, pbase + (size_t)r0 * wp + c1);
          rd[q] = load_texel(planes, pbase + (size_t)r1 * wp + c1);
          const bool x0 = in && ix >= 0 && ix < wp, x1 = in && ix + 1 >= 0 && ix + 1 < wp;
          const bool y0 = pi.iy >= 0, y1 = pi.iy + 1 < hp;
          valid |= ((x0 && y0 ? 1u : 0u) | (x0 && y1 ? 2u : 0u) | (x1 && y0 ? 4u : 0u) | (x1 && y1 ? 8u : 0u))
                   << (q * 4);
        }
      }
    };
    // branch free: entries past the window go to a trash slot behind the buffer (a branch
    // here would split the loop into blocks the compiler then schedules across)
    auto store = [&](int buf, int k) {
      const PlaneInfo pi = pinfo[k];
      float4* w = win + buf * WS;
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        if (q * nt >= pi.len) break;                       // uniform: the window is shorter
        const int i0 = tid + q * nt;
        const int i = i0 < pi.len ? i0 : (BIL ? W / 2 : W);
        const uint32_t m = valid >> (q * 4);
        if constexpr (BUF) {
          (void)m;
          if constexpr (U8) reinterpret_cast<uint2*>(w)[i] = codes_to_half4(praw[q]);
          else if constexpr (RAW) reinterpret_cast<uint2*>(w)[i] = praw[q];
          else w[i] = ra[q];
        } else if constexpr (RAW) {
          if constexpr (U8) reinterpret_cast<uint2*>(w)[i] = codes_to_half4(keep_if((m & 1u) != 0u, praw[q]));
          else reinterpret_cast<uint2*>(w)[i] = keep_if((m & 1u) != 0u, praw[q]);
        } else if constexpr (!BIL) {
          w[i] = keep_if((m & 1u) != 0u, ra[q]);
        } else {
          const float4 t0 = lerp4(keep_if((m & 1u) != 0u, ra[q]), keep_if((m & 2u) != 0u, rb[q]), pi.wy);
          const float4 t1 = lerp4(keep_if((m & 4u) != 0u, rc[q]), keep_if((m & 8u) != 0u, rd[q]), pi.wy);
          w[2 * i] = t0;
          w[2 * i + 1] = make_float4(t1.x - t0.x, t1.y - t0.y, t1.z - t0.z, t1.w - t0.w);
        }
      }
    };
    {
      fetch(slist[0]);
      store(0, slist[0]);
      __syncthreads();
      for (int n = 0; n < nvalid; ++n) {
        const int k = __builtin_amdgcn_readfirstlane(slist[n]);
        const bool more = n + 1 < nvalid;
        if (more) fetch(slist[n + 1]);
        const int f0 = __builtin_amdgcn_readfirstlane(pinfo[k].f0);
        const int len = __builtin_amdgcn_readfirstlane(pinfo[k].len);
        const float* crow = ct + (size_t)(kb + k) * V + v0;
        float Cv[G];
#pragma unroll
        for (int j = 0; j < G; ++j) Cv[j] = crow[j];          // scalar loads, one wait
        const float bxr = pt[kb + k].x * xr;
        const float xmin = (float)f0, xmax = (float)(f0 + len) - 0.5f;
        const char* wbytes = reinterpret_cast<const char*>(win) + (n & 1) * (WS * 16) -
                             (ptrdiff_t)f0 * (ptrdiff_t)(BIL ? 32 : (int)sizeof(LT));
#pragma unroll
        for (int j0 = 0; j0 < G; j0 += kSub) {
          // views in sub-blocks: kSub LDS reads in flight, then their blends (bounds live registers)
          float4 sv[kSub];
#pragma unroll
          for (int jj = 0; jj < kSub; ++jj) {
            const int j = j0 + jj;
            // the clamp is a no-op for fitting windows and holds a whole-row window's
            // samples on its zero guards
            const float X = __builtin_amdgcn_fmed3f(bxr + Cv[j], xmin, xmax);
            const int ix = cvt_flr(X);
            if (!BIL) {
              sv[jj] = lds_texel<LT>(wbytes + (ptrdiff_t)ix * (ptrdiff_t)sizeof(LT));
            } else {
              const float w = __builtin_amdgcn_fractf(X);
              const char* e = wbytes + (ptrdiff_t)ix * 32;
              const float4 t = *reinterpret_cast<const float4*>(e);
              const float4 dd = *reinterpret_cast<const float4*>(e + 16);
              sv[jj] = make_float4(fmaf(w, dd.x, t.x), fmaf(w, dd.y, t.y), fmaf(w, dd.z, t.z), fmaf(w, dd.w, t.w));
            }
          }
#pragma unroll
          for (int jj = 0; jj < kSub; ++jj) {
            const int j = j0 + jj;
            const float w = U8 ? Tr[j] * (1.0f / 255.0f) : Tr[j];
            Qr[j] = fmaf(w, sv[jj].x, Qr[j]);
            Qg[j] = fmaf(w, sv[jj].y, Qg[j]);
            Qb[j] = fmaf(w, sv[jj].z, Qb[j]);
            Tr[j] = fmaf(-w, sv[jj].w, Tr[j]);
          }
          // blend this sub-block before the next one's LDS reads are issued: bounds the
          // live sample registers (occupancy) instead of holding all G samples at once
#pragma unroll
          for (int jj = 0; jj < kSub; ++jj)
            asm volatile("" ::"v"(Qr[j0 + jj]), "v"(Qg[j0 + jj]), "v"(Qb[j0 + jj]), "v"(Tr[j0 + jj]) : "memory");
          __builtin_amdgcn_sched_barrier(0);
        }
        if (more) store((n + 1) & 1, slist[n + 1]);
        __syncthreads();
      }
    }
  }
  if (tid < seg_len && x < a.nx && !wave_done) {
    OT* out = static_cast<OT*>(a.out);
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (j < nv) store_pixel(out, ((size_t)a.perm[v0 + j] * a.ny + y) * a.nx + x, Qr[j], Qg[j], Qb[j], Tr[j]);
  }
}

// ---------------------------------------------------------------------------------------
// One-wave kernel: a work-group is one wave, 64 output pixels of row y (lane = pixel) for a
// group of G views that share dy, the G views' (Q, T) in registers; tiles dealt to the XCDs
// as in the row kernel.  It takes the segments whose every window fits kWaveWin entries
// (wave_fits; the row kernel takes the others).  A single wave needs no barrier: its LDS
// operations complete in order.  Plane windows are derived 64 at a time across the lanes
// and read out (readlane) when a plane is processed; the next plane's window is in flight
// in registers (buffer loads over the plane row: zero outside it) while this one is
// sampled, and the window buffers alternate, so a sample is floor(X) - f0 with no clamp.
//   nearest  : win[i] = texel f0 + i (FP16 and UNORM8 planes as FP16, others float32)
//   bilinear : win[2i] = t(f0 + i), win[2i+1] = t(f0 + i + 1) - t(f0 + i), t the row pair
//              blended vertically by the plane's weight wy
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ float4 wave_texel(__amdgpu_buffer_rsrc_t r, int ix);
template <>
__device__ __forceinline__ float4 wave_texel<float>(__amdgpu_buffer_rsrc_t r, int ix) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (uint32_t)ix * 16u, 0, 0));
}
template <>
__device__ __forceinline__ float4 wave_texel<__half>(__amdgpu_buffer_rsrc_t r, int ix) {
  const uint2 u = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, (uint32_t)ix * 8u, 0, 0));
  const float2 f = __half22float2(*reinterpret_cast<const __half2*>(&u.x));
  const float2 h = __half22float2(*reinterpret_cast<const __half2*>(&u.y));
  return make_float4(f.x, f.y, h.x, h.y);
}
template <>
__device__ __forceinline__ float4 wave_texel<__hip_bfloat16>(__amdgpu_buffer_rsrc_t r, int ix) {
  const uint2 u = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, (uint32_t)ix * 8u, 0, 0));
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                     __uint_as_float(u.y & 0xffff0000u));
}
template <>
__device__ __forceinline__ float4 wave_texel<uint8_t>(__amdgpu_buffer_rsrc_t r, int ix) {
  const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, (uint32_t)ix * 4u, 0, 0);
  constexpr float s = 1.0f / 255.0f;
  return make_float4((float)(u & 0xffu) * s, (float)((u >> 8) & 0xffu) * s, (float)((u >> 16) & 0xffu) * s,
                     (float)(u >> 24) * s);
}

template <typename PT, typename OT, int G, bool BIL>
__device__ __forceinline__ void composite_wave_tile(const CompositeArgs& a, int nseg, int lg, GF4 __restrict__ pt,
                                                   GF1 __restrict__ ct, GF2 __restrict__ pm) {
  // LDS texels: FP16 for FP16 / UNORM8 nearest windows (UNORM8 as codes 0..255), else float32
  using LT = typename std::conditional<BIL, float4, typename LdsTexel<PT>::type>::type;
  constexpr bool RAW = !std::is_same<LT, float4>::value;
  constexpr bool U8 = RAW && std::is_same<PT, uint8_t>::value;
  using RT = typename std::conditional<U8, uint32_t, typename std::conditional<RAW, uint2, float4>::type>::type;
  constexpr int E = BIL ? kWaveWin / 2 : kWaveWin;          // window entries
  constexpr int PF = E / 64;                                 // entries each lane fetches
  constexpr int kTB = std::is_same<PT, float>::value ? 16 : (std::is_same<PT, uint8_t>::value ? 4 : 8);
  __shared__ LT win[2][(BIL ? 2 : 1) * E + 2];              // (+2: the split halves' spacing)
  // Float32 nearest windows (FP32 planes, and BF16 planes widened to float32) are held as
  // two arrays of 8-byte halves, (r, g) at entries [0, E) and (b, a) kHalf entries on: a
  // sample is two ds_read_b64 at one address (the second through the instruction's
  // offset), which meet far fewer bank conflicts than one ds_read_b128 of neighbouring
  // texels.
  constexpr bool SPLIT = !RAW && !BIL;
  constexpr int kSubW = SPLIT && std::is_same<PT, float>::value && G % 8 == 0 ? 8 : kSub;
  constexpr int kHalf = E + 2;                               // float2 entries to the (b, a) half
  // the scalars of the arguments in registers: the asm memory barriers of the sample
  // loop would otherwise reload them when the arguments live in global memory
  const int aK = a.K, ahp = a.hp, awp = a.wp, anx = a.nx;
  const float acx = a.c.cx, acy = a.c.cy;
  const int gi = lg % a.n_groups, rest = lg / a.n_groups;
  const int y = rest / nseg, xs0 = (rest % nseg) * 64;
  const uint32_t gd = a.vgroup[gi];
  const int v0 = gd & 0xffu;
  const int nv = gd >> 8;
  pt += (size_t)gi * aK;
  pm += (size_t)gi * aK;
  if (!wave_fits<BIL>(a, pt, pm, xs0, y)) {                // the row kernel's segment
    if (threadIdx.x == 0 && a.spill) *a.spill = 1u;
    return;
  }
  const int lane = threadIdx.x;
  const int x = xs0 + lane;
  // lanes past the row's end sample at their own x (results dropped)
  const float xr = (float)x - acx, yr = (float)y - acy;
  const float xr_lo = (float)xs0 - acx, xr_hi = (float)(xs0 + 63) - acx;
  const int S = ct_stride(a.n_views);
  const char* planes = static_cast<const char*>(a.planes);
  const size_t plane_bytes = (size_t)ahp * awp * kTB;

  // plane windows, 64 at a time (lane i: plane kb + i); the planes sampled are the set bits
  // per lane: its plane's window start f0 (22-bit signed) and length (at most E) in one
  // word, so a plane's window takes one readlane less
  int my_fl = 0, my_iy = 0;
  float my_wy = 0.0f;
  auto batch = [&](int kb) -> uint64_t {
    const int k = kb + lane;
    int f0 = 0, len = 0, iy = 0;
    float wy = 0.0f;
    if (k < aK) {
      const float4 p = ld4(pt + k);
      const float2 cr = ld2(pm + k);
      const float Y = p.y * yr + p.z;
      const float fy0 = floorf(Y);
      wy = BIL ? Y - fy0 : 0.0f;
      iy = (int)fy0;
      bool ok = p.w != 0.0f && iy >= (BIL ? -1 : 0) && iy < ahp;
      const float lo = floorf(p.x * xr_lo + cr.x);
      const float hi = floorf(p.x * xr_hi + cr.y) + (BIL ? 1.0f : 0.0f);
      ok = ok && hi >= 0.0f && lo <= (float)(awp - 1);   // else transparent texels only
      f0 = ok ? (int)lo : 0;
      len = ok ? (int)(hi - lo) + 1 : 0;                   // <= E: wave_fits
    }
    my_fl = (f0 & 0x3fffff) | (len << 22);
    my_iy = iy;
    my_wy = wy;
    return __builtin_amdgcn_ballot_w64(len > 0);
  };
  int kb = 0;
  uint64_t mask = batch(0);
  auto next = [&](int& k, int& f0, int& len, int& iy, float& wy) {
    while (mask == 0) {
      kb += 64;
      if (kb >= aK) return false;
      mask = batch(kb);
    }
    const int i = __builtin_ctzll(mask);
    mask &= mask - 1;
    k = kb + i;
    const int fl = __builtin_amdgcn_readlane(my_fl, i);
    f0 = (fl << 10) >> 10;
    len = (int)((uint32_t)fl >> 22);
    iy = __builtin_amdgcn_readlane(my_iy, i);
    wy = BIL ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_wy), i)) : 0.0f;
    return true;
  };
  // buffer resource over row iy of plane k (a row outside the plane: no records, zeros)
  auto row = [&](int k, int iy) {
    const bool in = iy >= 0 && iy < ahp;
    const char* base = planes + (size_t)k * plane_bytes + (size_t)(in ? iy : 0) * awp * kTB;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), (short)0, in ? awp * kTB : 0, 0x00020000);
  };
  // window fetch into registers (nearest: raw texels; bilinear: the four corners)
  RT rn[BIL ? 1 : PF];
  float4 rc[BIL ? PF : 1][4];
  auto fetch = [&](int k, int f0, int len, int iy) {
    const auto r0 = row(k, iy);
    const auto r1 = row(k, iy + 1);
    // (texel f0 + lane + 64 q at byte (f0 + lane) kTB + 64 q kTB: one offset, the q steps
    // in the loads' immediate offsets; unsigned wrap-around keeps it exact)
    const uint32_t vo = (uint32_t)(f0 + lane) * (uint32_t)kTB;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      if (q * 64 >= len) break;                            // wave uniform
      const int ix = f0 + lane + q * 64;
      const uint32_t o = vo + (uint32_t)(q * 64 * kTB);
      if constexpr (!BIL) {
        if constexpr (U8) rn[q] = (RT)__builtin_amdgcn_raw_buffer_load_b32(r0, o, 0, 0);
        else if constexpr (RAW) rn[q] = __builtin_bit_cast(RT, __builtin_amdgcn_raw_buffer_load_b64(r0, o, 0, 0));
        else if constexpr (std::is_same<PT, float>::value)
          rn[q] = __builtin_bit_cast(RT, __builtin_amdgcn_raw_buffer_load_b128(r0, o, 0, 0));
        else rn[q] = __builtin_bit_cast(RT, wave_texel<PT>(r0, ix));
      } else {
        // (texel ix + 1 through an offset the compiler cannot relate to ix's: it would merge
        // the two loads into one wider load, which the range check zeroes as a whole at the
        // row's start)
        int ix1 = ix + 1;
        asm volatile("" : "+v"(ix1));
        rc[q][0] = wave_texel<PT>(r0, ix);
        rc[q][1] = wave_texel<PT>(r1, ix);
        rc[q][2] = wave_texel<PT>(r0, ix1);
        rc[q][3] = wave_texel<PT>(r1, ix1);
      }
    }
  };
  auto store = [&](LT* w, int len, float wy) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      if (q * 64 >= len) break;
      // entries past the window's end (i >= len) land in the buffer's unread tail
      const int i = lane + q * 64;
      if constexpr (SPLIT) {
        float2* w2 = reinterpret_cast<float2*>(w);
        const float4 t = __builtin_bit_cast(float4, rn[q]);
        w2[i] = make_float2(t.x, t.y);
        w2[kHalf + i] = make_float2(t.z, t.w);
      } else if constexpr (!BIL) {
        if constexpr (U8) w[i] = codes_to_half4(rn[q]);
        else w[i] = rn[q];
      } else {
        const float4 t0 = lerp4(rc[q][0], rc[q][1], wy);
        const float4 t1 = lerp4(rc[q][2], rc[q][3], wy);
        w[2 * i] = t0;
        w[2 * i + 1] = make_float4(t1.x - t0.x, t1.y - t0.y, t1.z - t0.z, t1.w - t0.w);
      }
    }
  };

  float Qr[G], Qg[G], Qb[G], Tr[G];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    Qr[j] = Qg[j] = Qb[j] = 0.0f;
    Tr[j] = 1.0f;
  }
  int k, f0, len, iy;
  float wy;
  bool have = next(k, f0, len, iy, wy);
  if (have) fetch(k, f0, len, iy);
  int buf = 0;
  while (have) {
    store(win[buf], len, wy);                              // this plane's window (fetched before)
    const int kc = k, f0c = f0;
    const float bxr = *(CF1)(pt + kc) * xr;
    const CF1 crow = (CF1)(ct + (size_t)kc * S + v0);
    float Cv[G];
#pragma unroll
    for (int j = 0; j < G; ++j) Cv[j] = crow[j];
    have = next(k, f0, len, iy, wy);
    if (have) fetch(k, f0, len, iy);                       // the next one, in flight meanwhile
    const char* wb = reinterpret_cast<const char*>(win[buf]) - (ptrdiff_t)f0c * (ptrdiff_t)(BIL ? 32 : SPLIT ? 8 : (int)sizeof(LT));
    // views in blocks of kSubW: the block's LDS reads all in flight, then its blends
#pragma unroll
    for (int j0 = 0; j0 < G; j0 += kSubW) {
      float4 sv[kSubW];
#pragma unroll
      for (int jj = 0; jj < kSubW; ++jj) {
        const float X = bxr + Cv[j0 + jj];
        const int ix = cvt_flr(X);
        if constexpr (SPLIT) {
          const char* e = wb + (ptrdiff_t)ix * 8;
          const float2 rg = *reinterpret_cast<const float2*>(e);
          const float2 ba = *reinterpret_cast<const float2*>(e + kHalf * 8);
          sv[jj] = make_float4(rg.x, rg.y, ba.x, ba.y);
        } else if constexpr (!BIL) {
          sv[jj] = lds_texel<LT>(wb + (ptrdiff_t)ix * (ptrdiff_t)sizeof(LT));
        } else {
          const float w = __builtin_amdgcn_fractf(X);
          const char* e = wb + (ptrdiff_t)ix * 32;
          const float4 t = *reinterpret_cast<const float4*>(e);
          const float4 dd = *reinterpret_cast<const float4*>(e + 16);
          sv[jj] = make_float4(fmaf(w, dd.x, t.x), fmaf(w, dd.y, t.y), fmaf(w, dd.z, t.z), fmaf(w, dd.w, t.w));
        }
      }
#pragma unroll
      for (int jj = 0; jj < kSubW; ++jj) {
        const int j = j0 + jj;
        const float w = U8 ? Tr[j] * (1.0f / 255.0f) : Tr[j];
        Qr[j] = fmaf(w, sv[jj].x, Qr[j]);
        Qg[j] = fmaf(w, sv[jj].y, Qg[j]);
        Qb[j] = fmaf(w, sv[jj].z, Qb[j]);
        Tr[j] = fmaf(-w, sv[jj].w, Tr[j]);
      }
      // (the block's blends before the next block's reads: bounds the live sample registers)
#pragma unroll
      for (int jj = 0; jj < kSubW; ++jj)
        asm volatile("" ::"v"(Qr[j0 + jj]), "v"(Qg[j0 + jj]), "v"(Qb[j0 + jj]), "v"(Tr[j0 + jj]) : "memory");
      __builtin_amdgcn_sched_barrier(0);
    }
    buf ^= 1;
  }
  if (x < anx) {
    OT* out = static_cast<OT*>(a.out);
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (j < nv) store_pixel(out, ((size_t)a.perm[v0 + j] * a.ny + y) * a.nx + x, Qr[j], Qg[j], Qb[j], Tr[j]);
  }
}

// One wave per 64-pixel segment of one scene; tile lg of `total` is dealt to the XCDs in
// contiguous runs (work-group w runs on XCD w mod 8), so the view groups and segments of
// one output row, which stage the same plane rows, share an L2.
template <typename PT, typename OT, int G, bool BIL>
__global__ __launch_bounds__(64) void composite_wave(CompositeArgs a, int nseg, int total,
                                                     const float4* __restrict__ pt, const float* __restrict__ ct,
                                                     const float2* __restrict__ pm) {
  const int wg = blockIdx.x;
  const int per = (total + 7) / 8;
  const int lg = (wg % 8) * per + wg / 8;
  if (lg >= total) return;                                 // whole work-group: grid padded to 8 per
  composite_wave_tile<PT, OT, G, BIL>(a, nseg, lg, (GF4)pt, (GF1)ct, (GF2)pm);
}

// The tiles of several scenes' composites in one launch: jobs [0 .. n) in a device array,
// start[j] = the first tile of job j in the launch's tile list (start[n] tiles in all).  A
// tile's job is found by a scan of the starts; tiles are dealt to the XCDs as above.
struct JobStarts {
  int32_t n;
  int32_t start[kMaxJobs + 1];
};

// Jobs differ in cost per tile (their plane counts), so the tiles go to the XCDs in
// 2^kJobShift blocks of consecutive tiles, block B on XCD B mod 8 (a block still holds the
// view groups and segments of about one output row): every XCD gets a share of every job.
constexpr int kJobShift = 9;

inline int64_t job_grid(int64_t total) {
  const int64_t C = std::max<int64_t>(1, total >> kJobShift);
  return ((total + 8 * C + 7) / 8) * 8;
}

template <typename PT, typename OT, int G, bool BIL>
__global__ __launch_bounds__(64) void composite_wave_jobs(const CompositeJob* __restrict__ jobs, JobStarts js) {
  const int total = js.start[js.n];
  const int C = max(1, total >> kJobShift);
  const int wg = blockIdx.x, jw = wg >> 3, xw = wg & 7;
  const int q = jw / C;
  const int lg = (q * 8 + xw) * C + (jw - q * C);
  if (lg >= total) return;
  int j = 0;
  while (j + 1 < js.n && lg >= js.start[j + 1]) ++j;
  const CompositeJob& jb = jobs[j];
  composite_wave_tile<PT, OT, G, BIL>(jb.a, jb.nseg, lg - js.start[j], (GF4)jb.pt, (GF1)jb.ct, (GF2)jb.pm);
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

// ---------------------------------------------------------------------------------------
// Backward of the composite (Eq. 7 over operator).  With Q = sum_k T_k c_k,
// T_{k+1} = T_k (1 - a_k) and cotangents g = dL/dQ, g_T = dL/dT_final:
//   dL/dc_k = T_k g,   dL/da_k = -T_k U_{k+1},   U_k = g . c_k + (1 - a_k) U_{k+1},  U_K = g_T
// (U_k = g . R_k + g_T S_k folds the colour R and transmittance S behind plane k into one
// scalar), evaluated back to front; a sample's cotangent goes to its texels through the
// transposed interpolation weights.
//
// One work-group is one wave: a segment of 64 output pixels of row y for a group of up to
// G views that share dy (lane = pixel, the G views in registers), tiles dealt to the XCDs as
// in the forward.  A single wave needs no barrier: its LDS operations complete in order.
// Transmittance is recomputed, not stored: sweep 1 (front to back, alpha only) finds per
// (pixel, view) the last plane m whose incoming transmittance T_m is at least kTinyT and
// keeps T_m; sweep 2 (back to front) recovers T_k = T_{k+1} / (1 - a_k) for k < m (exact up
// to rounding: T_{k+1} >= kTinyT there, a normal number, and 1 - a_k > 0) and gives planes
// behind m no gradient (below kTinyT |g|), while U keeps the colour behind them.
// Per plane the wave stages the window of the plane row its samples fall in (bilinear: the
// two rows blended vertically): sweep 1 its alpha, sweep 2 its texels, beside two LDS
// accumulators of the window.  A sample adds its cotangent (bilinear: its two weighted
// parts, one after the other) to an accumulator with a plain read-modify-write: x -> texel
// is monotone with slope bx, so lanes L or more apart never share a texel when L bx > 1.
// For L <= 2 (bx > 0.505, the usual case) even lanes update one accumulator and odd lanes
// the other, all in one instruction; otherwise the lanes update the first in L phases of
// lanes L apart.  The window is then added to the plane gradient with one global atomic
// per texel channel (windows of other rows, segments and view groups overlap it).
// ---------------------------------------------------------------------------------------
constexpr int kBwdWin = 128;          // texels of an LDS window chunk
constexpr int kBwdPf = kBwdWin / 64;  // window entries each lane fetches
constexpr float kTinyT = 1e-30f;
constexpr int kBufFlags = 0x00020000; // buffer resource: raw dword access, range checked

struct BwdInfo {
  float bx, wy;
  int32_t iy, f0, len;                // len 0: the plane is skipped (invalid, or wholly outside)
  int32_t phases;                     // L: lanes L apart never share a texel
};

// texel ix of a plane row through a buffer resource over that row: zero outside the row
// (the hardware's range check, also for ix < 0, whose offset wraps far past the row)
template <typename T>
__device__ __forceinline__ float4 buf_texel(__amdgpu_buffer_rsrc_t r, int ix);
template <>
__device__ __forceinline__ float4 buf_texel<float>(__amdgpu_buffer_rsrc_t r, int ix) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (uint32_t)ix * 16u, 0, 0));
}
template <>
__device__ __forceinline__ float4 buf_texel<__half>(__amdgpu_buffer_rsrc_t r, int ix) {
  const uint2 u = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, (uint32_t)ix * 8u, 0, 0));
  const __half2 lo = *reinterpret_cast<const __half2*>(&u.x), hi = *reinterpret_cast<const __half2*>(&u.y);
  const float2 f = __half22float2(lo), h = __half22float2(hi);
  return make_float4(f.x, f.y, h.x, h.y);
}
template <>
__device__ __forceinline__ float4 buf_texel<__hip_bfloat16>(__amdgpu_buffer_rsrc_t r, int ix) {
  const uint2 u = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, (uint32_t)ix * 8u, 0, 0));
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                     __uint_as_float(u.y & 0xffff0000u));
}

// alpha (A = 1 - T) of texel ix of a plane row, likewise
template <typename T>
__device__ __forceinline__ float buf_alpha(__amdgpu_buffer_rsrc_t r, int ix);
template <>
__device__ __forceinline__ float buf_alpha<float>(__amdgpu_buffer_rsrc_t r, int ix) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (uint32_t)ix * 16u + 12u, 0, 0));
}
template <>
__device__ __forceinline__ float buf_alpha<__half>(__amdgpu_buffer_rsrc_t r, int ix) {
  const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, (uint32_t)ix * 8u + 4u, 0, 0);
  return __half2float(__ushort_as_half((unsigned short)(u >> 16)));
}
template <>
__device__ __forceinline__ float buf_alpha<__hip_bfloat16>(__amdgpu_buffer_rsrc_t r, int ix) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (uint32_t)ix * 8u + 4u, 0, 0) & 0xffff0000u);
}

// FAST: the form for work-groups whose every window fits one chunk and whose planes all
// have L <= 2 (bx > 0.505); the general form takes the other work-groups.  Both are
// launched over every work-group, and each returns at once from the work-groups of the other.
template <typename PT, int G, bool BIL, bool FAST>
__global__ __launch_bounds__(64) void composite_rows_bwd(CompositeArgs a, int nseg, int total,
                                                         const float4* __restrict__ pt, const float* __restrict__ ct,
                                                         const float2* __restrict__ pm,
                                                         const float4* __restrict__ d_out, float* __restrict__ d_planes) {
  __shared__ float4 win[kBwdWin];                          // sweep 1: alpha (as floats); sweep 2: texels
  // sweep 2: cotangent accumulators (fast form: two, the second kBwdWin texels on)
  constexpr int kAcc = FAST ? 2 : 1;
  __shared__ float4 acc[kAcc * kBwdWin];
  __shared__ float tmL[G * 64];                            // T_m of view slot j at [j][lane]
  float* winA = reinterpret_cast<float*>(win);
  const int wg = blockIdx.x;
  const int per = (total + 7) / 8;
  const int lg = (wg % 8) * per + wg / 8;
  if (lg >= total) return;                                 // whole work-group: grid padded to 8 per
  const int gi = lg % a.n_groups, rest = lg / a.n_groups;
  const int y = rest / nseg, seg = rest % nseg;
  const uint32_t gd = a.vgroup[gi];
  const int v0 = gd & 0xffu;                               // group's first position in perm
  const int nv = gd >> 8;
  pt += (size_t)gi * a.K;
  pm += (size_t)gi * a.K;
  const int lane = threadIdx.x;
  const int xs0 = seg * 64;
  const int x = xs0 + lane;
  const bool xin = x < a.nx;
  // Every lane samples at its own x, also past the row's end (a pixel with a zero cotangent,
  // so its updates add zero), and every view slot of the group is sampled: the slots past a
  // short group's end read the table's padded positions (within the window the table's
  // per-group extents cover) with zero cotangents.  So the per-view code has no branches.
  const float xr = (float)x - a.c.cx, yr = (float)y - a.c.cy;
  const float xr_lo = (float)xs0 - a.c.cx, xr_hi = (float)(xs0 + 63) - a.c.cx;
  const int S = ct_stride(a.n_views);
  const size_t plane_elems = (size_t)a.hp * a.wp;
  constexpr int kTB = sizeof(PT) * 4;                      // bytes per texel
  const char* planes = static_cast<const char*>(a.planes);
  // a window wider than the LDS buffer is processed in chunks of kBwdWin texels (bilinear:
  // overlapping by one, so each sample's two texels lie in the chunk that owns its first)
  constexpr int kStride = BIL ? kBwdWin - 1 : kBwdWin;

  // Plane windows, 64 planes at a time: lane i derives the window of plane kb + i (the
  // texels every sample of the wave falls in), its row and weight; a plane's fields are read
  // out of its lane (wave uniform) when it is processed.  The planes with a window are the
  // set bits of the batch mask.
  int my_f0 = 0, my_len = 0, my_iy = 0;
  float my_wy = 0.0f;
  bool my_slow = false;                                    // needs the general form
  auto batch = [&](int kb) -> uint64_t {
    const int k = kb + lane;
    int f0 = 0, len = 0, iy = 0;
    float wy = 0.0f;
    bool slow = false;
    if (k < a.K) {
      const float4 p = pt[k];                              // (bx, by, Cy, L)
      const float2 cr = pm[k];                             // least and greatest Cx of the group
      bool ok = p.w != 0.0f;
      if (!BIL) {
        iy = (int)floorf(p.y * yr + p.z);
        ok = ok && iy >= 0 && iy < a.hp;
      } else {
        const float Y = p.y * yr + p.z;
        const float fy0 = floorf(Y);
        wy = Y - fy0;
        iy = (int)fy0;
        ok = ok && iy >= -1 && iy < a.hp;
      }
      // X = bx xr + C is monotone in xr and C (each rounding is monotone), so the samples
      // of the wave lie in [floor(X(xr_lo, cmin)), floor(X(xr_hi, cmax))] (+1 bilinear)
      const float lo = floorf(p.x * xr_lo + cr.x);
      const float hi = floorf(p.x * xr_hi + cr.y) + (BIL ? 1.0f : 0.0f);
      // a window wholly outside the row samples only transparent texels: a = 0 leaves T
      // and U unchanged and texels outside the plane get no gradient, so the plane is
      // skipped; the window is clipped to the columns [-kBwdWin, wp + kBwdWin) (samples
      // outside the plane read zero texels there) so its length stays an int
      ok = ok && hi >= 0.0f && lo <= (float)(a.wp - 1);
      const float lc = fmaxf(lo, (float)-kBwdWin), hc = fminf(hi, (float)(a.wp + kBwdWin - 1));
      f0 = ok ? (int)lc : 0;
      len = ok ? (int)(hc - lc) + 1 : 0;
      slow = ok && (len > kBwdWin || p.w > 2.0f);
    }
    my_f0 = f0;
    my_len = len;
    my_iy = iy;
    my_wy = wy;
    my_slow = slow;
    return __builtin_amdgcn_ballot_w64(len > 0);
  };
  // the form this work-group takes: the fast one when no plane needs the general one
  {
    bool slow = false;
    for (int kb = 0; kb < a.K; kb += 64) {
      batch(kb);
      slow = slow || __builtin_amdgcn_ballot_w64(my_slow) != 0;
    }
    if (slow == FAST) return;
  }
  auto plane_at = [&](int i, int k) {
    BwdInfo b;
    b.f0 = __builtin_amdgcn_readlane(my_f0, i);
    b.len = __builtin_amdgcn_readlane(my_len, i);
    b.iy = __builtin_amdgcn_readlane(my_iy, i);
    b.wy = BIL ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_wy), i)) : 0.0f;
    const float4 p = pt[k];
    b.bx = p.x;
    b.phases = (int)p.w;
    return b;
  };
  int kb = 0;
  uint64_t mask = 0;
  // the next plane with a window front to back (sweep 1) or back to front (sweep 2)
  auto next_fwd = [&](int& k, BwdInfo& b) {
    while (mask == 0) {
      kb += 64;
      if (kb >= a.K) return false;
      mask = batch(kb);
    }
    const int i = __builtin_ctzll(mask);
    mask &= mask - 1;
    k = kb + i;
    b = plane_at(i, k);
    return true;
  };
  auto next_bwd = [&](int& k, BwdInfo& b) {
    while (mask == 0) {
      kb -= 64;
      if (kb < 0) return false;
      mask = batch(kb);
    }
    const int i = 63 - __builtin_clzll(mask);
    mask &= ~(1ull << i);
    k = kb + i;
    b = plane_at(i, k);
    return true;
  };
  // buffer resources over rows iy and iy + 1 of plane k (a row outside the plane: zero
  // records, so every read returns zero)
  auto row_rsrc = [&](int k, int iy, int width_bytes) {
    const bool in = iy >= 0 && iy < a.hp;
    const char* base = planes + ((size_t)k * plane_elems + (size_t)(in ? iy : 0) * a.wp) * kTB;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), (short)0, in ? width_bytes : 0, kBufFlags);
  };
  // Chunks of a window (the fast form: one).  Of a window of several chunks, chunk
  // [c0, c0 + clen) owns the samples whose texel (bilinear: first texel) lies in
  // [c0, c0 + clen) ([c0, c0 + clen - 1)); the others read a safe texel and update nothing.
  auto chunks = [&](const BwdInfo& b) {
    return FAST || b.len <= kBwdWin ? 1 : 1 + (b.len - kBwdWin + kStride - 1) / kStride;
  };
  auto owned = [&](int& ix, int c0, uint32_t lim) {
    if (FAST) return true;
    const bool own = (uint32_t)(ix - c0) < lim;
    ix = own ? ix : c0;
    return own;
  };
  float cv[G];                                             // the plane's Cx of each view slot
  auto load_cx = [&](int k) {
    const float* crow = ct + (size_t)k * S + v0;
#pragma unroll
    for (int j = 0; j < G; ++j) cv[j] = crow[j];
  };

  float T[G], Tm[G];
  int m[G];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    T[j] = 1.0f;
    Tm[j] = 1.0f;
    m[j] = -1;
  }

  // ---- sweep 1: front to back over alpha, last plane with incoming T >= kTinyT ----------
  // The next plane's first alpha chunk is fetched into registers while this one is sampled.
  float pa0[kBwdPf], pa1[BIL ? kBwdPf : 1];
  auto fetch_alpha = [&](const BwdInfo& b, int k, int c0) {
    const auto r0 = row_rsrc(k, b.iy, a.wp * kTB);
    const auto r1 = row_rsrc(k, b.iy + 1, a.wp * kTB);
#pragma unroll
    for (int q = 0; q < kBwdPf; ++q) {
      pa0[q] = buf_alpha<PT>(r0, c0 + lane + q * 64);
      if (BIL) pa1[BIL ? q : 0] = buf_alpha<PT>(r1, c0 + lane + q * 64);
    }
  };
  auto store_alpha = [&](const BwdInfo& b, int clen) {
#pragma unroll
    for (int q = 0; q < kBwdPf; ++q) {
      const int i = lane + q * 64;
      const float v = BIL ? fmaf(b.wy, pa1[BIL ? q : 0] - pa0[q], pa0[q]) : pa0[q];
      if (i < clen) winA[i] = v;
    }
  };
  auto pass1 = [&](int k, float bxr, int c0, int clen) {
    const float* wa = winA - c0;
    const uint32_t lim = (uint32_t)(clen - (BIL ? 1 : 0));
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const float X = bxr + cv[j];
      float al;
      bool own;
      if (!BIL) {
        int ix = cvt_flr(X);
        own = owned(ix, c0, lim);
        al = wa[ix];
      } else {
        const float fx = floorf(X), wx = X - fx;
        int ix = cvt_flr(fx);
        own = owned(ix, c0, lim);
        al = fmaf(wx, wa[ix + 1] - wa[ix], wa[ix]);
      }
      const bool live = own && T[j] >= kTinyT;
      m[j] = live ? k : m[j];
      Tm[j] = live ? T[j] : Tm[j];
      const float Tn = fmaf(-T[j], al, T[j]);
      T[j] = own ? Tn : T[j];
    }
  };
  {
    kb = 0;
    mask = batch(0);
    int k = 0;
    BwdInfo b{};
    bool have = next_fwd(k, b);
    if (have) fetch_alpha(b, k, b.f0);
    while (have) {
      const float bxr = b.bx * xr;
      load_cx(k);
      const int nch = chunks(b);
      int kn = 0;
      BwdInfo bn{};
      bool have_n = false;
      for (int c = 0; c < nch; ++c) {
        const int c0 = b.f0 + c * kStride, clen = min(kBwdWin, b.len - c * kStride);
        if (c > 0) fetch_alpha(b, k, c0);
        store_alpha(b, clen);                              // chunk 0: the prefetched one
        if (c == nch - 1) {
          have_n = next_fwd(kn, bn);
          if (have_n) fetch_alpha(bn, kn, bn.f0);
        }
        pass1(k, bxr, c0, clen);
      }
      k = kn;
      b = bn;
      have = have_n;
    }
  }

  // ---- sweep 2: back to front, gradients of the planes at or before m -------------------
  // T_m goes to LDS (read at plane m only) and m + 1 to 16-bit halves, two views a register.
  uint32_t mp[(G + 1) / 2];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    tmL[j * 64 + lane] = Tm[j];
    const uint32_t h = (uint32_t)(m[j] + 1);
    mp[j / 2] = (j & 1) ? (mp[j / 2] | (h << 16)) : h;
  }
  float4 g[G];
  float Tc[G], U[G];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    g[j] = (xin && j < nv) ? d_out[((size_t)a.perm[v0 + j] * a.ny + y) * a.nx + x] : make_float4(0.f, 0.f, 0.f, 0.f);
    Tc[j] = 0.0f;                                          // stays 0 behind m
    U[j] = g[j].w;                                         // U_K = g_T
  }
  for (int i = lane; i < kAcc * kBwdWin; i += 64) acc[i] = make_float4(0.f, 0.f, 0.f, 0.f);   // flushes re-zero
  float4 pr0[kBwdPf], pr1[BIL ? kBwdPf : 1];
  auto fetch = [&](const BwdInfo& b, int k, int c0) {
    const auto r0 = row_rsrc(k, b.iy, a.wp * kTB);
    const auto r1 = row_rsrc(k, b.iy + 1, a.wp * kTB);
#pragma unroll
    for (int q = 0; q < kBwdPf; ++q) {
      pr0[q] = buf_texel<PT>(r0, c0 + lane + q * 64);
      if (BIL) pr1[BIL ? q : 0] = buf_texel<PT>(r1, c0 + lane + q * 64);
    }
  };
  auto store = [&](const BwdInfo& b, int clen) {
#pragma unroll
    for (int q = 0; q < kBwdPf; ++q) {
      const int i = lane + q * 64;
      const float4 v = BIL ? lerp4(pr0[q], pr1[BIL ? q : 0], b.wy) : pr0[q];
      if (i < clen) win[i] = v;
    }
  };
  // the accumulators' sum added to the plane gradient (rows iy, iy + 1 split by wy for
  // bilinear) through buffer atomics over the row: columns outside the plane are dropped by
  // the range check.  One channel word per lane: consecutive lanes add consecutive words, so
  // an atomic instruction covers whole cache lines.  The accumulators are re-zeroed.
  auto flush = [&](const BwdInfo& b, int k, int c0, int clen) {
    const bool in0 = b.iy >= 0 && b.iy < a.hp, in1 = BIL && b.iy + 1 < a.hp;   // iy >= -1
    char* gp = reinterpret_cast<char*>(d_planes) + (size_t)k * a.hp * a.wp * 16;
    const auto g0 = __builtin_amdgcn_make_buffer_rsrc(gp + (size_t)(in0 ? b.iy : 0) * a.wp * 16, (short)0,
                                                      in0 ? a.wp * 16 : 0, kBufFlags);
    const auto g1 = __builtin_amdgcn_make_buffer_rsrc(gp + (size_t)(in1 ? b.iy + 1 : 0) * a.wp * 16, (short)0,
                                                      in1 ? a.wp * 16 : 0, kBufFlags);
    // word i = 4 t + c of the window (channel c of texel t) at lane i mod 64, summed over the
    // accumulators.  The whole buffers are read, then cleared (past the window they hold
    // zeros), so that no read waits on another.
    float* af = reinterpret_cast<float*>(acc) + lane;
    constexpr int kIt = kBwdWin * 4 / 64;
    float v[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      v[it] = af[64 * it];
      if (kAcc == 2) v[it] += af[64 * it + 4 * kBwdWin];
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      af[64 * it] = 0.0f;
      if (kAcc == 2) af[64 * it + 4 * kBwdWin] = 0.0f;
    }
    const uint32_t off = (uint32_t)c0 * 16u + (uint32_t)lane * 4u;
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      if (v[it] != 0.0f) {                                 // (zero past the window)
        if (!BIL) {
          __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(v[it], g0, off + 256u * it, 0, 0);
        } else {
          __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32((1.0f - b.wy) * v[it], g0, off + 256u * it, 0, 0);
          __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(b.wy * v[it], g1, off + 256u * it, 0, 0);
        }
      }
    }
  };
  // Sample pass of sweep 2 over a window chunk.
  // Fast form: x -> texel is monotone and lanes 2 apart never share a texel, so even lanes
  // update the first accumulator and odd lanes the second, all in one read-modify-write.
  // General form: samples owned by the chunk update the first in L phases (phase of lane l:
  // ph).
  float4* const acc_lane = acc + (FAST && (lane & 1) ? kBwdWin : 0);
  auto pass2 = [&](int k, float bxr, int c0, int clen, int L, int ph) {
    const float4* wt = win - c0;
    float4* ac = acc_lane - c0;
    const uint32_t lim = (uint32_t)(clen - (BIL ? 1 : 0));
    // Lanes update texels other lanes read and write next, which the compiler cannot see:
    // an empty asm with a memory clobber after every update keeps the LDS operations in
    // program order (one wave executes them in order, so no wait is needed).
    // adds s e to accumulator entry i (one rounding per channel)
    auto scatter = [&](int i, float sc, const float4& e, bool own) {
      auto rmw = [&]() {
        float4 v = ac[i];
        v.x = fmaf(sc, e.x, v.x);
        v.y = fmaf(sc, e.y, v.y);
        v.z = fmaf(sc, e.z, v.z);
        v.w = fmaf(sc, e.w, v.w);
        ac[i] = v;
      };
      if (FAST) {
        rmw();
        asm volatile("" ::: "memory");
      } else {
        for (int p = 0; p < L; ++p) {
          if (own && ph == p) rmw();
          asm volatile("" ::: "memory");
        }
      }
    };
    // the texel (bilinear: the blend) of view slot j, its column ix, weight wx, ownership
    auto sample = [&](int j, int& ix, float& wx, bool& own) {
      const float X = bxr + cv[j];
      wx = 0.0f;
      if (!BIL) {
        ix = cvt_flr(X);
        own = owned(ix, c0, lim);
        return wt[ix];
      }
      const float fx = floorf(X);
      wx = X - fx;
      ix = cvt_flr(fx);
      own = owned(ix, c0, lim);
      return lerp4(wt[ix], wt[ix + 1], wx);
    };
    int ixn;
    float wxn;
    bool ownn;
    float4 sn = sample(0, ixn, wxn, ownn);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int ix = ixn;
      const float wx = wxn;
      const bool own = ownn;
      const float4 s = sn;
      if (j + 1 < G) sn = sample(j + 1, ixn, wxn, ownn);   // read ahead of this view's updates
      const float om = 1.0f - s.w;
      const float gc = fmaf(g[j].z, s.z, fmaf(g[j].y, s.y, g[j].x * s.x));
      // T_k: kept at m, recovered from T_{k+1} before it (reciprocal to ~1 ulp; 1 - a > 0
      // there), 0 behind it (Tc = 0; the clamp keeps 0 / (1 - a) finite)
      float Tk = Tc[j] * __builtin_amdgcn_rcpf(fmaxf(om, kTinyT));
      const uint32_t mj = (j & 1) ? (mp[j / 2] >> 16) : (mp[j / 2] & 0xffffu);
      const bool at_m = mj == (uint32_t)(k + 1);
      if (__builtin_amdgcn_ballot_w64(at_m) != 0) {        // wave uniform
        const float tm = tmL[j * 64 + lane];
        Tk = at_m ? tm : Tk;
      }
      // the sample's cotangent: Tk (g_r, g_g, g_b, -U)
      const float4 d = make_float4(g[j].x, g[j].y, g[j].z, -U[j]);
      float Un = fmaf(om, U[j], gc);
      // (an empty asm pins the update here: sunk below the scatters, it would keep every
      // view's texel live across them)
      asm volatile("" : "+v"(Un));
      Tc[j] = own ? Tk : Tc[j];
      U[j] = own ? Un : U[j];
      if (!BIL) {
        scatter(ix, Tk, d, own);
      } else {
        scatter(ix, (1.0f - wx) * Tk, d, own);
        scatter(ix + 1, wx * Tk, d, own);
      }
    }
  };
  {
    kb = ((a.K - 1) / 64) * 64;
    mask = batch(kb);
    int k = 0;
    BwdInfo b{};
    bool have = next_bwd(k, b);
    if (have) fetch(b, k, b.f0);
    while (have) {
      const float bxr = b.bx * xr;
      load_cx(k);
      const int L = b.phases;
      // lane l updates in phase l mod L (general form): lane / L = (lane mul) >> 16 for lanes < 64
      int ph = 0;
      if (!FAST) {
        const uint32_t mul = (uint32_t)ceilf(65536.0f * __builtin_amdgcn_rcpf((float)L));
        ph = lane - L * (int)(((uint32_t)lane * mul) >> 16);
      }
      const int nch = chunks(b);
      int kn = 0;
      BwdInfo bn{};
      bool have_n = false;
      for (int c = 0; c < nch; ++c) {
        const int c0 = b.f0 + c * kStride, clen = min(kBwdWin, b.len - c * kStride);
        if (c > 0) fetch(b, k, c0);
        store(b, clen);                                    // chunk 0: the prefetched one
        if (c == nch - 1) {
          have_n = next_bwd(kn, bn);
          if (have_n) fetch(bn, kn, bn.f0);
        }
        pass2(k, bxr, c0, clen, L, ph);
        flush(b, k, c0, clen);
      }
      k = kn;
      b = bn;
      have = have_n;
    }
  }
}

__global__ void zero_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// threads of a row work-group, and whether the whole-row window fits its buffer and fetch
// Threads of a row work-group for its segment of seg pixels: one per pixel, and enough
// (up to kRowThreads) for the fetch of the whole-row fallback, wp + 4 entries at kPrefetch
// per thread (half for bilinear); the threads past the segment only fetch.
int row_threads(const CompositeArgs& a, int* seg_out) {
  // segments of kRowThreads pixels (a multiple of 64: the one-wave kernel's segments nest)
  const int seg = std::min(kRowThreads, (a.nx + 63) / 64 * 64);
  const int per_thread = a.interp == LF_BILINEAR ? kPrefetch / 2 : kPrefetch;
  const int need = std::min((a.wp + 4 + per_thread - 1) / per_thread, kRowThreads);
  if (seg_out) *seg_out = seg;
  return (std::max(seg, need) + 63) / 64 * 64;
}

bool rows_fit(const CompositeArgs& a) {
  const bool bil = a.interp == LF_BILINEAR;
  const int entries = a.wp + 4;
  const int per_thread = bil ? kPrefetch / 2 : kPrefetch;
  return entries <= (bil ? kWin / 2 : kWin) && entries <= per_thread * row_threads(a, nullptr);
}

// Views that share dy, as classes in the order of their first view, each class's views in
// index order: perm lists them class by class, cls_end[c] is where class c ends in perm.
int dy_classes(CompositeArgs& a, int* cls_end) {
  bool placed[LF_MAX_VIEWS] = {};
  int n = 0, nc = 0;
  for (int v = 0; v < a.n_views; ++v) {
    if (placed[v]) continue;
    for (int u = v; u < a.n_views; ++u) {
      if (!placed[u] && a.dy[u] == a.dy[v]) {
        placed[u] = true;
        a.perm[n++] = (uint8_t)u;
      }
    }
    cls_end[nc++] = n;
  }
  return nc;
}

// Row-kernel cost of groups of G: work-groups per row times their per-view work plus a
// fixed per-plane part worth about four views.
int group_cost(const int* cls_end, int nc, int G) {
  int cost = 0;
  for (int c = 0, s = 0; c < nc; s = cls_end[c++]) cost += (cls_end[c] - s + G - 1) / G * (G + 4);
  return cost;
}

// Cuts every class into runs of at most G views: a.vgroup / a.n_groups.
void fill_groups(CompositeArgs& a, const int* cls_end, int nc, int G) {
  int g = 0;
  for (int c = 0, s = 0; c < nc; s = cls_end[c++])
    for (int p = s; p < cls_end[c]; p += G) a.vgroup[g++] = (uint16_t)(p | (std::min(G, cls_end[c] - p) << 8));
  a.n_groups = g;
}

// Table of composite coefficients: pt [groups][K] float4, ct [K][ct_stride(V)] float, then
// pm [groups][K] float2 (at most one view group per view).
size_t align_256(size_t v) { return (v + 255) & ~(size_t)255; }

void table_parts(void* table, int K, int V, float4** pt, float** ct, float2** pm) {
  char* t = static_cast<char*>(table);
  const size_t o_ct = align_256((size_t)K * V * 16), o_pm = o_ct + align_256((size_t)K * ct_stride(V) * 4);
  *pt = reinterpret_cast<float4*>(t);
  *ct = reinterpret_cast<float*>(t + o_ct);
  *pm = reinterpret_cast<float2*>(t + o_pm);
}

void launch_table(const CompositeArgs& a, float4* pt, float* ct, float2* pm, hipStream_t s, int slots = 0) {
  const int n = a.K * ct_stride(a.n_views);
  hipLaunchKernelGGL(coeff_table, dim3((n + 255) / 256), dim3(256), 0, s, a, pt, ct, pm, slots);
}

template <typename PT, typename OT, bool BIL>
hipError_t launch_rows(const CompositeArgs& a, int G, const float4* pt, const float* ct, const float2* pm,
                       hipStream_t s) {
  int seg;
  const int threads = row_threads(a, &seg);
  const int nseg = (a.nx + seg - 1) / seg;
  const size_t lds = (size_t)2 * kWinStride * 16;
  const int total = a.n_groups * nseg * a.ny;
  const dim3 grid((unsigned)(((total + 7) / 8) * 8)), block(threads);
  const int nseg64 = (a.nx + 63) / 64;
  const int total64 = a.n_groups * nseg64 * a.ny;
  const dim3 grid64((unsigned)(((total64 + 7) / 8) * 8)), block64(64);
  // the one-wave kernel over every 64-pixel segment, then the row kernel over every
  // segment of seg pixels: each takes the 64-pixel segments that are its own
  auto both = [&](auto wave, auto rows) {
    if (a.tile != 256) hipLaunchKernelGGL(wave, grid64, block64, 0, s, a, nseg64, total64, pt, ct, pm);
    hipLaunchKernelGGL(rows, grid, block, lds, s, a, seg, nseg, total, pt, ct, pm);
  };
  switch (G) {
    case 4: both(composite_wave<PT, OT, 4, BIL>, composite_rows<PT, OT, 4, BIL>); break;
    case 8: both(composite_wave<PT, OT, 8, BIL>, composite_rows<PT, OT, 8, BIL>); break;
    case 12: both(composite_wave<PT, OT, 12, BIL>, composite_rows<PT, OT, 12, BIL>); break;
    case 24: both(composite_wave<PT, OT, 24, BIL>, composite_rows<PT, OT, 24, BIL>); break;
    default: both(composite_wave<PT, OT, 16, BIL>, composite_rows<PT, OT, 16, BIL>); break;
  }
  return hipGetLastError();
}

template <typename PT, typename OT>
hipError_t dispatch_interp(const CompositeArgs& a, bool rows, int G, const float4* pt, const float* ct,
                           const float2* pm, hipStream_t s) {
  if (rows)
    return a.interp == LF_BILINEAR ? launch_rows<PT, OT, true>(a, G, pt, ct, pm, s)
                                   : launch_rows<PT, OT, false>(a, G, pt, ct, pm, s);
  const int64_t n = (int64_t)a.n_views * a.ny * a.nx;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (a.interp == LF_BILINEAR)
    hipLaunchKernelGGL((composite_general<PT, OT, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((composite_general<PT, OT, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename PT>
hipError_t dispatch_out(const CompositeArgs& a, bool rows, int G, const float4* pt, const float* ct,
                        const float2* pm, hipStream_t s) {
  return a.out_dtype == LF_F16 ? dispatch_interp<PT, __half>(a, rows, G, pt, ct, pm, s)
                               : dispatch_interp<PT, float>(a, rows, G, pt, ct, pm, s);
}

template <typename PT, int G>
void launch_rows_bwd_g(const CompositeArgs& a, int nseg, int total, const float4* pt, const float* ct,
                       const float2* pm, const float4* go, float* d_planes, hipStream_t s) {
  const dim3 grid((unsigned)(((total + 7) / 8) * 8)), blk(64);
  // both forms over every work-group: each takes the work-groups that are its own
  if (a.interp == LF_BILINEAR) {
    hipLaunchKernelGGL((composite_rows_bwd<PT, G, true, true>), grid, blk, 0, s, a, nseg, total, pt, ct, pm, go, d_planes);
    hipLaunchKernelGGL((composite_rows_bwd<PT, G, true, false>), grid, blk, 0, s, a, nseg, total, pt, ct, pm, go, d_planes);
  } else {
    hipLaunchKernelGGL((composite_rows_bwd<PT, G, false, true>), grid, blk, 0, s, a, nseg, total, pt, ct, pm, go, d_planes);
    hipLaunchKernelGGL((composite_rows_bwd<PT, G, false, false>), grid, blk, 0, s, a, nseg, total, pt, ct, pm, go, d_planes);
  }
}

template <typename PT>
hipError_t launch_rows_bwd(const CompositeArgs& a, int G, const float4* pt, const float* ct, const float2* pm,
                           const float* d_out, float* d_planes, hipStream_t s) {
  const int nseg = (a.nx + 63) / 64;
  const int total = a.n_groups * nseg * a.ny;
  const float4* go = reinterpret_cast<const float4*>(d_out);
  if (G == 16) launch_rows_bwd_g<PT, 16>(a, nseg, total, pt, ct, pm, go, d_planes, s);
  else if (G == 12) launch_rows_bwd_g<PT, 12>(a, nseg, total, pt, ct, pm, go, d_planes, s);
  else launch_rows_bwd_g<PT, 8>(a, nseg, total, pt, ct, pm, go, d_planes, s);
  return hipGetLastError();
}

}  // namespace

int view_groups(CompositeArgs& a, int G) {
  int cls_end[LF_MAX_VIEWS];
  const int nc = dy_classes(a, cls_end);
  fill_groups(a, cls_end, nc, G);
  return a.n_groups;
}

size_t composite_table_bytes(int K, int n_views) {
  // at most one view group per view; the last 256 bytes hold the spill flag
  return align_256((size_t)K * n_views * 16) + align_256((size_t)K * ct_stride(n_views) * 4) +
         align_256((size_t)K * n_views * 8) + 256;
}

uint32_t* table_spill(void* table, int K, int n_views) {
  return reinterpret_cast<uint32_t*>(static_cast<char*>(table) + composite_table_bytes(K, n_views) - 256);
}

namespace {

// The view-group size G and kernel form of a composite (the row kernels, or the per-pixel
// kernel when rows is false); fills a's view groups for G.
void composite_plan(CompositeArgs& a, int* G_out, bool* rows_out) {
  int cls_end[LF_MAX_VIEWS];
  const int nc = dy_classes(a, cls_end);
  int G = 16, best = group_cost(cls_end, nc, 16);
  for (int g : {12, 8, 4}) {
    const int c = group_cost(cls_end, nc, g);
    if (c < best) { G = g; best = c; }
  }
  // The row kernel needs the clamped whole-row fallback to fit the window buffer and the
  // fetch of one work-group (kPrefetch entries per thread, half of them for bilinear).  It
  // is taken while its cost stays below about four units per view: measured on MI355X
  // (512 x 512 views, 64 planes, 45 views) a cost unit takes 0.006 ms nearest / 0.013 ms
  // bilinear and the per-pixel kernel 0.025 / 0.05 ms per view, so quilts with several views
  // per dy take the row kernel and lists of all-distinct dy the per-pixel one.
  // LF_COMPOSITE_KERNEL=rows|general overrides the choice (tuning and tests).
  const char* kern = getenv("LF_COMPOSITE_KERNEL");
  bool rows = best <= 4 * a.n_views;
  if (kern && std::strcmp(kern, "rows") == 0) rows = true;
  if (kern && std::strcmp(kern, "general") == 0) rows = false;
  rows = rows && rows_fit(a);
  // an explicit group (autotuned) wins; else the LF_COMPOSITE_GROUP tuning override
  if (a.group == 4 || a.group == 8 || a.group == 12 || a.group == 16 || a.group == 24) {
    G = a.group;
  } else if (const char* e = getenv("LF_COMPOSITE_GROUP")) {
    const int g = atoi(e);
    if (g == 4 || g == 8 || g == 12 || g == 16 || g == 24) G = g;
  }
  // an explicit tile (autotuned) wins; else LF_COMPOSITE_TILE=256 sends every segment to the
  // row kernel
  if (a.tile != 64 && a.tile != 256) {
    const char* t = getenv("LF_COMPOSITE_TILE");
    a.tile = t && atoi(t) == 256 ? 256 : 64;
  }
  fill_groups(a, cls_end, nc, G);
  *G_out = G;
  *rows_out = rows;
}

template <typename PT, typename OT, int G, bool BIL>
void launch_jobs_wave(const CompositeJob* jobs, const JobStarts& js, hipStream_t s) {
  const dim3 grid((unsigned)job_grid(js.start[js.n]));
  hipLaunchKernelGGL((composite_wave_jobs<PT, OT, G, BIL>), grid, dim3(64), 0, s, jobs, js);
}

template <typename PT, typename OT, bool BIL>
void launch_jobs_g(const CompositeJob* jobs, const JobStarts& js, int G, hipStream_t s) {
  switch (G) {
    case 4: launch_jobs_wave<PT, OT, 4, BIL>(jobs, js, s); break;
    case 8: launch_jobs_wave<PT, OT, 8, BIL>(jobs, js, s); break;
    case 12: launch_jobs_wave<PT, OT, 12, BIL>(jobs, js, s); break;
    case 24: launch_jobs_wave<PT, OT, 24, BIL>(jobs, js, s); break;
    default: launch_jobs_wave<PT, OT, 16, BIL>(jobs, js, s); break;
  }
}

template <typename PT, typename OT>
void launch_jobs_interp(const CompositeJob* jobs, const JobStarts& js, const CompositeKey& k, hipStream_t s) {
  if (k.interp == LF_BILINEAR) launch_jobs_g<PT, OT, true>(jobs, js, k.group, s);
  else launch_jobs_g<PT, OT, false>(jobs, js, k.group, s);
}

template <typename PT>
void launch_jobs_out(const CompositeJob* jobs, const JobStarts& js, const CompositeKey& k, hipStream_t s) {
  if (k.out_dtype == LF_F16) launch_jobs_interp<PT, __half>(jobs, js, k, s);
  else launch_jobs_interp<PT, float>(jobs, js, k, s);
}

// The row kernel alone over one job's segments (those that do not fit a wave).
template <typename PT, typename OT, bool BIL>
hipError_t launch_rows_only(const CompositeArgs& a, int G, const float4* pt, const float* ct, const float2* pm,
                            hipStream_t s) {
  CompositeArgs b = a;
  b.tile = 64;
  int seg;
  const int threads = row_threads(b, &seg);
  const int nseg = (b.nx + seg - 1) / seg;
  const size_t lds = (size_t)2 * kWinStride * 16;
  const int total = b.n_groups * nseg * b.ny;
  const dim3 grid((unsigned)(((total + 7) / 8) * 8)), block(threads);
  switch (G) {
    case 4: hipLaunchKernelGGL((composite_rows<PT, OT, 4, BIL>), grid, block, lds, s, b, seg, nseg, total, pt, ct, pm); break;
    case 8: hipLaunchKernelGGL((composite_rows<PT, OT, 8, BIL>), grid, block, lds, s, b, seg, nseg, total, pt, ct, pm); break;
    case 12: hipLaunchKernelGGL((composite_rows<PT, OT, 12, BIL>), grid, block, lds, s, b, seg, nseg, total, pt, ct, pm); break;
    case 24: hipLaunchKernelGGL((composite_rows<PT, OT, 24, BIL>), grid, block, lds, s, b, seg, nseg, total, pt, ct, pm); break;
    default: hipLaunchKernelGGL((composite_rows<PT, OT, 16, BIL>), grid, block, lds, s, b, seg, nseg, total, pt, ct, pm); break;
  }
  return hipGetLastError();
}

template <typename PT, typename OT>
hipError_t rows_only_interp(const CompositeJob& j, int G, hipStream_t s) {
  return j.a.interp == LF_BILINEAR ? launch_rows_only<PT, OT, true>(j.a, G, j.pt, j.ct, j.pm, s)
                                   : launch_rows_only<PT, OT, false>(j.a, G, j.pt, j.ct, j.pm, s);
}

template <typename PT>
hipError_t rows_only_out(const CompositeJob& j, int G, hipStream_t s) {
  return j.a.out_dtype == LF_F16 ? rows_only_interp<PT, __half>(j, G, s) : rows_only_interp<PT, float>(j, G, s);
}

}  // namespace

hipError_t composite_launch(CompositeArgs& a, void* table, hipStream_t s, Profiler* prof) {
  float4* pt;
  float* ct;
  float2* pm;
  table_parts(table, a.K, a.n_views, &pt, &ct, &pm);
  a.spill = table_spill(table, a.K, a.n_views);
  int G;
  bool rows;
  composite_plan(a, &G, &rows);
  if (rows) {
    PhaseScope ps(prof, LF_PHASE_COEFF, s);
    launch_table(a, pt, ct, pm, s, G);                     // every view slot is sampled
  }
  PhaseScope ps(prof, LF_PHASE_COMPOSITE, s);
  switch (a.plane_dtype) {
    case LF_F16: return dispatch_out<__half>(a, rows, G, pt, ct, pm, s);
    case LF_BF16: return dispatch_out<__hip_bfloat16>(a, rows, G, pt, ct, pm, s);
    case LF_U8: return dispatch_out<uint8_t>(a, rows, G, pt, ct, pm, s);
    default: return dispatch_out<float>(a, rows, G, pt, ct, pm, s);
  }
}

bool composite_job(CompositeArgs& a, void* table, CompositeJob* j, CompositeKey* key) {
  float4* pt;
  float* ct;
  float2* pm;
  table_parts(table, a.K, a.n_views, &pt, &ct, &pm);
  a.spill = table_spill(table, a.K, a.n_views);
  int G;
  bool rows;
  composite_plan(a, &G, &rows);
  if (!rows || a.tile == 256) return false;
  a.group = G;                                             // the table's slots and the kernel's
  j->a = a;
  j->pt = pt;
  j->ct = ct;
  j->pm = pm;
  j->nseg = (a.nx + 63) / 64;
  j->tiles = a.n_groups * j->nseg * a.ny;
  *key = CompositeKey{a.plane_dtype, a.out_dtype, a.interp, G};
  return true;
}

hipError_t composite_job_table(const CompositeJob& j, hipStream_t s) {
  launch_table(j.a, const_cast<float4*>(j.pt), const_cast<float*>(j.ct), const_cast<float2*>(j.pm), s, j.a.group);
  return hipGetLastError();
}

hipError_t composite_jobs_launch(const CompositeJob* jobs, const CompositeJob* jobs_host, int n, const CompositeKey& k,
                                 hipStream_t s) {
  if (n < 1 || n > kMaxJobs) return hipErrorInvalidValue;
  JobStarts js;
  js.n = n;
  js.start[0] = 0;
  for (int i = 0; i < n; ++i) js.start[i + 1] = js.start[i] + jobs_host[i].tiles;
  if (js.start[n] > 0) {
    switch (k.plane_dtype) {
      case LF_F16: launch_jobs_out<__half>(jobs, js, k, s); break;
      case LF_BF16: launch_jobs_out<__hip_bfloat16>(jobs, js, k, s); break;
      case LF_U8: launch_jobs_out<uint8_t>(jobs, js, k, s); break;
      default: launch_jobs_out<float>(jobs, js, k, s); break;
    }
  }
  hipError_t e = hipGetLastError();
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    switch (k.plane_dtype) {
      case LF_F16: e = rows_only_out<__half>(jobs_host[i], k.group, s); break;
      case LF_BF16: e = rows_only_out<__hip_bfloat16>(jobs_host[i], k.group, s); break;
      case LF_U8: e = rows_only_out<uint8_t>(jobs_host[i], k.group, s); break;
      default: e = rows_only_out<float>(jobs_host[i], k.group, s); break;
    }
  }
  return e;
}

hipError_t composite_backward_launch(CompositeArgs& a, void* table, const float* d_out, float* d_planes,
                                    hipStream_t s, Profiler* prof) {
  float4* pt;
  float* ct;
  float2* pm;
  table_parts(table, a.K, a.n_views, &pt, &ct, &pm);
  // views per work-group (one wave, the views in registers): 16, or 8 / 12 (LF_BWD_GROUP);
  // 16 does the per-plane work (window staging, gradient atomics) for the most views
  int G = 16;
  if (const char* e = getenv("LF_BWD_GROUP"))
    if (atoi(e) == 8 || atoi(e) == 12) G = atoi(e);
  int cls_end[LF_MAX_VIEWS];
  const int nc = dy_classes(a, cls_end);
  fill_groups(a, cls_end, nc, G);
  {
    PhaseScope ps(prof, LF_PHASE_COEFF, s);
    launch_table(a, pt, ct, pm, s, G);
  }
  PhaseScope ps(prof, LF_PHASE_COMPOSITE_BWD, s);
  const int64_t np = (int64_t)a.K * a.hp * a.wp * 4;
  if (np > 0) hipLaunchKernelGGL(zero_f32, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, d_planes, np);
  switch (a.plane_dtype) {
    case LF_F16: return launch_rows_bwd<__half>(a, G, pt, ct, pm, d_out, d_planes, s);
    case LF_BF16: return launch_rows_bwd<__hip_bfloat16>(a, G, pt, ct, pm, d_out, d_planes, s);
    default: return launch_rows_bwd<float>(a, G, pt, ct, pm, d_out, d_planes, s);
  }
}

hipError_t plane_coeffs_launch(const CompositeArgs& a, float* bx, float* by, float* cx, float* cy,
                               float* cxn, float* cyn, hipStream_t s) {
  const int n = a.K * a.n_views;
  hipLaunchKernelGGL(plane_coeffs_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, bx, by, cx, cy, cxn, cyn);
  return hipGetLastError();
}

}  // namespace lf
