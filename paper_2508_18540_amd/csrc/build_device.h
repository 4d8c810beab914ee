// Device helpers shared by the Gaussian and voxel MPI builds.
#pragma once

#include <algorithm>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "build_internal.h"

namespace lf {

// Order-preserving map of a finite float to u32 (negative values flip all bits).
__device__ __forceinline__ uint32_t orderable(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float unorderable(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// Depth key (base-camera z) and reference-frustum test of a primitive centre, float32 in a
// fixed operation order ((r0 x + r1 y) + r2 z) + t, no fused multiply-add (the library is
// built with -ffp-contract=off).  Visible iff the values are finite, z_ref = key - D_fwd >
// z_near, |x_c| <= guard_x z_ref and |y_c| <= guard_y z_ref.
struct KeyCull {
  float xc, yc, key;
  bool vis;
};

__device__ __forceinline__ KeyCull key_and_cull(const Consts& c, float mx, float my, float mz) {
  KeyCull k;
  k.xc = ((c.R[0] * mx + c.R[1] * my) + c.R[2] * mz) + c.t[0];
  k.yc = ((c.R[3] * mx + c.R[4] * my) + c.R[5] * mz) + c.t[1];
  k.key = (((c.R[6] * mx + c.R[7] * my) + c.R[8] * mz) + c.t[2]) + 0.0f;
  const float zr = k.key - c.d_fwd;
  k.vis = isfinite(k.key) && isfinite(k.xc) && isfinite(k.yc) && zr > c.z_near && fabsf(k.xc) <= c.guard_x * zr &&
          fabsf(k.yc) <= c.guard_y * zr;
  return k;
}

// Tile count of an inclusive texel box (0 if empty).
__device__ __forceinline__ uint32_t box_tiles(int x0, int y0, int x1, int y1) {
  if (x1 < x0 || y1 < y0) return 0u;
  return (uint32_t)(((x1 >> kTileShift) - (x0 >> kTileShift) + 1) * ((y1 >> kTileShift) - (y0 >> kTileShift) + 1));
}

// Segments of a (tile, chunk) bucket of len entries: runs of kSegment entries, and one
// (empty) segment for an empty bucket, whose texels are still written.
__device__ __forceinline__ uint32_t seg_count(uint32_t len) { return len ? (len + kSegment - 1) / kSegment : 1u; }

// Chunk-major work-item order, (chunk, tile): a run of consecutive items is a band of tile
// rows of one plane.  A run of items dealt to one XCD then reads the records of the
// plane's Gaussians in that band (which several of its tiles share) once into that XCD's
// L2.  item_order(bidx) is the position of (tile, chunk) bucket bidx = tile K + chunk in
// this order, item_bucket its inverse.  (The tile-major order is bidx itself.)
__device__ __forceinline__ int64_t item_order(const BuildArgs& a, int64_t bidx) {
  return (bidx % a.K) * a.n_tiles + bidx / a.K;
}

__device__ __forceinline__ int64_t item_bucket(const BuildArgs& a, int64_t c) {
  return (c % a.n_tiles) * a.K + c / a.n_tiles;
}

// Work item of work-group wg when `total` items are dealt to the 8 XCDs (work-group wg runs
// on XCD wg mod 8) in 2^shift blocks of consecutive items, block B on XCD B mod 8: as the
// items run in item_order, a block is a band of neighbouring tiles of one plane, whose
// lists share Gaussians, so it reads the shared records from one L2, while the dense and
// sparse parts of the frame are spread over all XCDs.  Within an XCD its work-groups take
// its blocks' items in order.  The grid must hold xcd_grid(max_items, shift) work-groups
// (total <= max_items); work-groups past the items return.
__device__ __forceinline__ bool xcd_item(uint32_t wg, uint32_t total, int shift, uint32_t* item) {
  const uint32_t C = max(1u, total >> shift);              // items per block
  const uint32_t j = wg >> 3, x = wg & 7u;
  const uint32_t q = j / C, r = j - q * C;
  *item = (q * 8u + x) * C + r;
  return *item < total;
}

// Work-groups of a launch over at most max_items items dealt by xcd_item: with C <=
// max(1, max_items >> shift) items per block, XCD x holds ceil(blocks / 8) blocks of C, so
// the largest index used is below total + 8 C.
inline int64_t xcd_grid(int64_t max_items, int shift) {
  const int64_t C = std::max<int64_t>(1, max_items >> shift);
  return ((max_items + 8 * C + 7) / 8) * 8;
}

// Premultiplied RGBA texel store in the plane's storage type (round to nearest even).
template <typename T>
__device__ __forceinline__ void store_rgba(T* p, size_t i, float r, float g, float b, float al);

template <>
__device__ __forceinline__ void store_rgba<float>(float* p, size_t i, float r, float g, float b, float al) {
  reinterpret_cast<float4*>(p)[i] = make_float4(r, g, b, al);
}

template <>
__device__ __forceinline__ void store_rgba<__half>(__half* p, size_t i, float r, float g, float b, float al) {
  const __half2 lo = __floats2half2_rn(r, g), hi = __floats2half2_rn(b, al);
  uint2 u;
  u.x = *reinterpret_cast<const uint32_t*>(&lo);
  u.y = *reinterpret_cast<const uint32_t*>(&hi);
  reinterpret_cast<uint2*>(p)[i] = u;
}

__device__ __forceinline__ uint32_t bf16_rn(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

template <>
__device__ __forceinline__ void store_rgba<__hip_bfloat16>(__hip_bfloat16* p, size_t i, float r, float g, float b,
                                                           float al) {
  uint2 u;
  u.x = bf16_rn(r) | (bf16_rn(g) << 16);
  u.y = bf16_rn(b) | (bf16_rn(al) << 16);
  reinterpret_cast<uint2*>(p)[i] = u;
}

// UNORM8 code of a float32 value: round-to-nearest-even of 255 v, v clamped to [0, 1]
// (NaN -> 0).
__device__ __forceinline__ uint32_t unorm8_rn(float v) {
  const float c = fminf(fmaxf(v, 0.0f), 1.0f);
  return (uint32_t)__builtin_rintf(c * 255.0f);
}

template <>
__device__ __forceinline__ void store_rgba<uint8_t>(uint8_t* p, size_t i, float r, float g, float b, float al) {
  reinterpret_cast<uint32_t*>(p)[i] = unorm8_rn(r) | (unorm8_rn(g) << 8) | (unorm8_rn(b) << 16) | (unorm8_rn(al) << 24);
}

// Texel load of a plane in its storage type, widened to float32 (exactly; UNORM8 as
// code / 255 to float32 rounding).
template <typename T>
__device__ __forceinline__ float4 load_rgba(const T* p, size_t i);

template <>
__device__ __forceinline__ float4 load_rgba<float>(const float* p, size_t i) {
  return reinterpret_cast<const float4*>(p)[i];
}

template <>
__device__ __forceinline__ float4 load_rgba<__half>(const __half* p, size_t i) {
  const uint2 u = reinterpret_cast<const uint2*>(p)[i];
  const __half2 lo = *reinterpret_cast<const __half2*>(&u.x), hi = *reinterpret_cast<const __half2*>(&u.y);
  const float2 a = __half22float2(lo), b = __half22float2(hi);
  return make_float4(a.x, a.y, b.x, b.y);
}

template <>
__device__ __forceinline__ float4 load_rgba<__hip_bfloat16>(const __hip_bfloat16* p, size_t i) {
  const uint2 u = reinterpret_cast<const uint2*>(p)[i];
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                     __uint_as_float(u.y & 0xffff0000u));
}

template <>
__device__ __forceinline__ float4 load_rgba<uint8_t>(const uint8_t* p, size_t i) {
  const uint32_t u = reinterpret_cast<const uint32_t*>(p)[i];
  constexpr float s = 1.0f / 255.0f;
  return make_float4((float)(u & 0xffu) * s, (float)((u >> 8) & 0xffu) * s, (float)((u >> 16) & 0xffu) * s,
                     (float)(u >> 24) * s);
}

}  // namespace lf
