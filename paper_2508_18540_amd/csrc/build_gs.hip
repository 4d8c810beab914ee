// MPI build for 3D Gaussians (G2LF, Sec. 4.4; Alg. 1 steps 1-5) for gfx950.
//
//  preprocess  per Gaussian: float32 depth key and reference-frustum cull (exact op order,
//              shared with the oracle's float32 decision program), double-float projected
//              mean, float32 EWA covariance with the Eq. 8 dilation, conic in log2 units,
//              support box {o G >= 1/255} and its tile rectangle
//  sort        stable radix sort of (key, index): the (depth, index) order of Alg. 1
//  rank        chunk of every rank (quantile: floor(r K / N_vis); inverse depth: edge count)
//  chunks      chunk starts, counts and plane depths d_k (lower-median key)
//  emit        one (tile, Gaussian) entry per covered tile, written in rank order, keyed
//              (tile << chunk_bits) | chunk
//  tile sort   stable radix sort of the entries by the tile bits only: each tile's list stays
//              in rank order, so every (tile, chunk) bucket is a contiguous, depth-ordered
//              run whose start a binary search over the sorted keys finds
//  splat       one work-group per (tile, chunk): front-to-back blending of the bucket into
//              premultiplied RGBA (C, 1 - T) with alpha = min(0.99, o G), only where
//              o G >= 1/255, no early termination
#include <algorithm>
#include <cstdlib>

#include "build_device.h"
#include "sh_basis.h"
#include "dfloat.h"
#include "sort_internal.h"

namespace lf {
namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLog2AlphaMin = -7.994353436858858f;   // log2(1/255)
constexpr float kAlphaMax = 0.99f;

// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void preprocess_gs(BuildArgs a) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i0 < a.n;
  const int64_t i = in ? i0 : a.n - 1;
  const Consts& c = a.c;
  const float mx = a.means[3 * i], my = a.means[3 * i + 1], mz = a.means[3 * i + 2];
  if (!in) return;
  const KeyCull kc = key_and_cull(c, mx, my, mz);
  const bool vis = kc.vis;
  a.keys[i] = vis ? orderable(kc.key) : 0xffffffffu;
  a.vals[i] = (uint32_t)i;
  a.ntiles_i[i] = 0;
  if (a.chunk_of) a.chunk_of[i] = -1;
  if (!vis) return;

  // projected mean in double-float: p = R m + t, z = p_z - D_forward, mu = f' p / z + c'
  df px = two_prod(c.R[0], mx), py = two_prod(c.R[3], mx), pz = two_prod(c.R[6], mx);
  px = df_add(df_add(px, two_prod(c.R[1], my)), two_prod(c.R[2], mz));
  py = df_add(df_add(py, two_prod(c.R[4], my)), two_prod(c.R[5], mz));
  pz = df_add(df_add(pz, two_prod(c.R[7], my)), two_prod(c.R[8], mz));
  px = df_add_f(px, c.t[0]);
  py = df_add_f(py, c.t[1]);
  pz = df_add_f(pz, c.t[2]);
  const df z = df_add(pz, df{-c.d_fwd, -c.d_fwd_lo});
  const df mux = df_add_f(df_mul(df_div(px, z), df{c.fpx, c.fpx_lo}), c.cpx);
  const df muy = df_add_f(df_mul(df_div(py, z), df{c.fpy, c.fpy_lo}), c.cpy);

  // world covariance R(q) diag(e^{2l}) R(q)^T, camera rotation, EWA Jacobian (float32)
  float qw = a.quats[4 * i], qx = a.quats[4 * i + 1], qy = a.quats[4 * i + 2], qz = a.quats[4 * i + 3];
  const float qn = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= qn; qx *= qn; qy *= qn; qz *= qn;
  const float Rg[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                       2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                       2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
  const float s0 = expf(a.log_scales[3 * i]), s1 = expf(a.log_scales[3 * i + 1]), s2 = expf(a.log_scales[3 * i + 2]);
  // M = W Rg diag(s): columns are the scaled principal axes in camera space
  float M[9];
  for (int r = 0; r < 3; ++r) {
    const float w0 = c.R[3 * r], w1 = c.R[3 * r + 1], w2 = c.R[3 * r + 2];
    M[3 * r + 0] = (w0 * Rg[0] + w1 * Rg[3] + w2 * Rg[6]) * s0;
    M[3 * r + 1] = (w0 * Rg[1] + w1 * Rg[4] + w2 * Rg[7]) * s1;
    M[3 * r + 2] = (w0 * Rg[2] + w1 * Rg[5] + w2 * Rg[8]) * s2;
  }
  const float zf = z.hi;
  const float iz = 1.0f / zf;
  const float j00 = c.fpx * iz, j02 = -c.fpx * px.hi * iz * iz;
  const float j11 = c.fpy * iz, j12 = -c.fpy * py.hi * iz * iz;
  // rows of J M (2x3); Sigma' = (J M)(J M)^T + f' I
  float u[3], v[3];
  for (int k = 0; k < 3; ++k) {
    u[k] = j00 * M[k] + j02 * M[6 + k];
    v[k] = j11 * M[3 + k] + j12 * M[6 + k];
  }
  const float sa = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + c.f_dil;
  const float sb = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
  const float sc = (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) + c.f_dil;
  // determinant a c - b^2 with Kahan's compensated product difference, clamped at f'^2
  const float bb = sb * sb;
  const float det_raw = fmaf(sa, sc, -bb) + fmaf(-sb, sb, bb);
  const float det = fmaxf(det_raw, fmaxf(c.f_dil * c.f_dil, 1e-10f));
  const float idet = 1.0f / det;
  const float o = a.opacity[i];

  GRec r;
  r.mx_hi = mux.hi;
  r.my_hi = muy.hi;
  r.mx_lo = mux.lo;
  r.my_lo = muy.lo;
  // log2 of o G(d) = l2o + ca dx^2 + cb dx dy + cc dy^2
  r.ca = -0.5f * kLog2e * sc * idet;
  r.cb = kLog2e * sb * idet;
  r.cc = -0.5f * kLog2e * sa * idet;
  r.l2o = log2f(o);
  r.rgb[0] = a.rgb[3 * i];
  r.rgb[1] = a.rgb[3 * i + 1];
  r.rgb[2] = a.rgb[3 * i + 2];
  r.pad = 0.0f;
  r.x0 = r.y0 = 0;
  r.x1 = r.y1 = -1;
  // support box of {q <= 2 ln(255 o)}, widened by a 1e-3 relative margin
  const float r2 = 2.0f * (5.541263545158426f + logf(o));
  uint32_t nt = 0;
  if (r2 >= 0.0f) {
    const float hx = sqrtf(r2 * sa) * 1.001f + 1e-3f;
    const float hy = sqrtf(r2 * sc) * 1.001f + 1e-3f;
    const float fx0 = fmaxf(ceilf(mux.hi - hx), 0.0f), fx1 = fminf(floorf(mux.hi + hx), (float)(c.wp - 1));
    const float fy0 = fmaxf(ceilf(muy.hi - hy), 0.0f), fy1 = fminf(floorf(muy.hi + hy), (float)(c.hp - 1));
    if (fx0 <= fx1 && fy0 <= fy1) {
      r.x0 = (int)fx0;
      r.x1 = (int)fx1;
      r.y0 = (int)fy0;
      r.y1 = (int)fy1;
      nt = (uint32_t)(((r.x1 >> kTileShift) - (r.x0 >> kTileShift) + 1) *
                      ((r.y1 >> kTileShift) - (r.y0 >> kTileShift) + 1));
    }
  }
  a.rec[i] = r;
  a.ntiles_i[i] = nt;
}

// N_vis = number of visible keys: culled primitives carry the largest key and sort last, so
// the one rank whose key is visible and whose successor is not (or is the end) sets it.
// (The header starts at zero, which stays the answer when nothing is visible.)
__global__ __launch_bounds__(256) void find_nvis(BuildArgs a, const uint32_t* skeys) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n) return;
  if (skeys[r] != 0xffffffffu && (r + 1 == a.n || skeys[r + 1] == 0xffffffffu)) a.hdr->n_vis = r + 1;
}

// chunk of a visible key under inverse-depth binning: number of interior edges <= key
__device__ __forceinline__ int edge_count(const float* edges, int ne, float key) {
  int lo = 0, hi = ne;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (edges[mid] <= key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void rank_pass(BuildArgs a, const uint32_t* skeys, const uint32_t* svals) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n) return;
  const int64_t nvis = a.hdr->n_vis;
  if (r >= nvis) {
    a.ntiles_r[r] = 0;
    return;
  }
  const uint32_t idx = svals[r];
  int chunk;
  if (a.binning == LF_BIN_QUANTILE) chunk = (int)((r * (int64_t)a.K) / nvis);
  else chunk = edge_count(a.edges, a.K - 1, unorderable(skeys[r]));
  a.chunk_r[r] = (uint32_t)chunk;
  if (a.chunk_of) a.chunk_of[idx] = chunk;
  a.ntiles_r[r] = a.ntiles_i[idx];
}

// chunk_start[k] for k in [0, K]: first rank whose chunk is >= k
__device__ void chunk_start_of(const BuildArgs& a, const uint32_t* skeys, int k) {
  const int64_t nvis = a.hdr->n_vis;
  int64_t s;
  if (k == 0) s = 0;
  else if (k == a.K) s = nvis;
  else if (a.binning == LF_BIN_QUANTILE) s = ((int64_t)k * nvis + a.K - 1) / a.K;
  else {
    const float e = a.edges[k - 1];
    int64_t lo = 0, hi = nvis;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (unorderable(skeys[mid]) < e) lo = mid + 1;
      else hi = mid;
    }
    s = lo;
  }
  a.chunk_start[k] = s;
}

// plane depth d_k and primitive count of chunk k (reads the starts of other chunks)
__device__ void chunk_depth_of(const BuildArgs& a, const uint32_t* skeys, int k) {
  const int64_t s = a.chunk_start[k], cnt = a.chunk_start[k + 1] - s;
  if (a.chunk_count) a.chunk_count[k] = (int32_t)cnt;
  float d;
  if (a.binning == LF_BIN_INV_DEPTH) {
    d = a.dtab[k];
  } else if (cnt > 0) {
    d = unorderable(skeys[s + (cnt - 1) / 2]);               // lower median of the chunk
  } else if (s > 0) {
    // empty chunk: the depth of the previous non-empty chunk, the one holding rank s - 1
    const int64_t nvis = a.hdr->n_vis;
    const int kp = (int)(((s - 1) * a.K) / nvis);
    const int64_t sp = a.chunk_start[kp], cp = a.chunk_start[kp + 1] - sp;
    d = unorderable(skeys[sp + (cp - 1) / 2]);
  } else {
    d = a.d_focal32;
  }
  a.depth[k] = d;
}

// Chunk starts, then depths and counts, in one work-group (the barrier orders the two).
__global__ __launch_bounds__(1024) void chunk_table(BuildArgs a, const uint32_t* skeys) {
  for (int k = threadIdx.x; k <= a.K; k += blockDim.x) chunk_start_of(a, skeys, k);
  __syncthreads();
  for (int k = threadIdx.x; k < a.K; k += blockDim.x) chunk_depth_of(a, skeys, k);
}

// One (tile, Gaussian) entry per covered tile, written in rank order.  Work is balanced by
// output: block b writes entries [256 b, 256 b + 256) of the rank-ordered list, whatever
// ranks they come from (a Gaussian near the camera can cover hundreds of tiles).  The
// block's first rank comes from the offsets scan (heads), the block stages the offsets of
// its rank range in LDS, and each thread finds its entry's rank by binary search there (or
// in the global offsets when the range is too long to stage).  Block 0 also records the
// number of entries.  The entry value carries the Gaussian index
// in its low 28 bits and, in bits 28..31, which 8x8 quadrants of the tile its support box
// touches (bit = 2 * qy + qx).
constexpr int kEmitRanks = 512;
constexpr int64_t kCombineGroups = 8192;
constexpr int kKeyDigitBits = 8;    // key sort: four passes over a grid wide enough to fill the CUs
constexpr int kTileDigitBits = 10;  // tile sort: one pass over up to 1024 tiles (writes are reordered in LDS)

__device__ __forceinline__ int64_t last_le(const uint64_t* off, int64_t lo, int64_t hi, uint64_t v) {
  // last r in [lo, hi] with off[r] <= v (off is non-decreasing, off[lo] <= v)
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void emit_entries(BuildArgs a, const uint32_t* svals) {
  __shared__ uint64_t soff[kEmitRanks + 1];
  __shared__ int64_t srange[2];
  const uint64_t total = a.offsets[a.n];
  const int t = threadIdx.x;
  if (blockIdx.x == 0 && t == 0) {
    a.hdr->entries = (int64_t)total;
    a.hdr->capacity = a.capacity;
  }
  if (total > (uint64_t)a.capacity) {
    if (blockIdx.x == 0 && t == 0) atomicOr(&a.hdr->overflow, 1);
    return;
  }
  const uint64_t o0 = (uint64_t)blockIdx.x * 256;
  if (o0 >= total) return;
  const uint64_t olast = min(total, o0 + 256) - 1;
  // the rank holding entry o0 comes from the offsets scan; the one holding entry o0 + 256
  // (if any) bounds the rank of the last entry from above
  const int64_t r_lo = a.heads[blockIdx.x];
  if (t == 0) srange[1] = o0 + 256 < total ? (int64_t)a.heads[blockIdx.x + 1] : last_le(a.offsets, r_lo, a.n, olast);
  __syncthreads();
  const int64_t r_hi = srange[1];
  const int64_t nr = r_hi - r_lo + 1;
  const bool staged = nr <= kEmitRanks;
  if (staged)
    for (int i = t; i <= nr; i += 256) soff[i] = a.offsets[r_lo + i];
  __syncthreads();
  const uint64_t o = o0 + t;
  if (o > olast) return;
  int64_t r;
  uint64_t start;
  if (staged) {
    int lo = 0, hi = (int)nr - 1;                          // last j with soff[j] <= o
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (soff[mid] <= o) lo = mid;
      else hi = mid - 1;
    }
    r = r_lo + lo;
    start = soff[lo];
  } else {
    r = last_le(a.offsets, r_lo, r_hi, o);
    start = a.offsets[r];
  }
  const uint32_t idx = svals[r];
  const int4 g = *reinterpret_cast<const int4*>(reinterpret_cast<const char*>(a.rec) + (size_t)idx * a.rec_bytes);
  const uint32_t u = (uint32_t)(o - start);
  const int sx0 = g.x >> kTileShift, sw = (g.z >> kTileShift) - sx0 + 1;
  const int tx = sx0 + (int)(u % (uint32_t)sw), ty = (g.y >> kTileShift) + (int)(u / (uint32_t)sw);
  const int ox = tx << kTileShift, oy = ty << kTileShift;
  uint32_t mask = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int bx = ox + ((q & 1) << 3), by = oy + ((q >> 1) << 3);
    if (g.z >= bx && g.x <= bx + 7 && g.w >= by && g.y <= by + 7) mask |= 1u << q;
  }
  const uint32_t tile = (uint32_t)(ty * a.ntx + tx);
  a.ekeys[o] = (tile << a.chunk_bits) | a.chunk_r[r];
  a.evals[o] = idx | (mask << 28);
}

// Start of every (tile, chunk) bucket in the tile-sorted entry list: the first entry whose
// (tile, chunk) key is not below the bucket's.  bucket[n_buckets] = number of entries.
__global__ __launch_bounds__(256) void bucket_bounds(BuildArgs a, const uint32_t* sekeys, int64_t n_buckets) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > n_buckets) return;
  const int64_t ne = a.hdr->overflow ? 0 : min(a.hdr->entries, a.capacity);
  if (b == n_buckets) {
    a.bucket[b] = (uint32_t)ne;
    return;
  }
  const uint32_t key = ((uint32_t)(b / a.K) << a.chunk_bits) | (uint32_t)(b % a.K);
  int64_t lo = 0, hi = ne;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (sekeys[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  a.bucket[b] = (uint32_t)lo;
}

// ---------------------------------------------------------------------------------------
// Splat: one work-group per (tile, chunk) segment of at most kSegment = 256 entries.
// Wave w of the 256 threads owns the 8x8 texel block at ((w & 1) * 8, (w >> 1) * 8) of the
// 16x16 tile.  First every thread stages one entry's Gaussian record in LDS (one coalesced
// 64-byte load per Gaussian, shared by the four waves) and the work-group compacts, per
// quadrant, the entries whose support box touches it (stable, so depth order is kept).
// Then each wave walks its own list reading records from LDS (broadcast reads): no scalar
// memory traffic and no per-entry test on the critical path.
// ---------------------------------------------------------------------------------------
// Split every (tile, chunk) bucket into segments of at most kSegment entries: nseg per
// bucket, at its position in the work-item order (chunk-major: item_order, else the bucket
// index), and the number of partial-tile slots of split buckets (at the bucket index).
__global__ void bucket_segments(BuildArgs a, int64_t n_buckets, int chunk_major) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_buckets) return;
  const uint32_t ns = seg_count(a.bucket[b + 1] - a.bucket[b]);
  a.nseg[chunk_major ? item_order(a, b) : b] = ns;
  a.pcnt[b] = ns > 1 ? ns : 0u;
}

// One (bucket, segment) work item per segment, in the work-item order: thread c handles the
// bucket at position c.  The kernels that take the items need not know the order: they
// find a bucket's segment count from its bounds.
__global__ void emit_items(BuildArgs a, int64_t n_buckets, int chunk_major) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_buckets) return;
  const int64_t b = chunk_major ? item_bucket(a, c) : c;
  const uint32_t i0 = a.item_start[c], ns = a.item_start[c + 1] - i0;
  for (uint32_t s = 0; s < ns; ++s) a.items[i0 + s] = make_uint2((uint32_t)b, s);
  if (ns > 1) {
    // the partial slots of a split bucket: the first names the bucket, the others nothing
    const uint32_t p0 = a.pslot[b];
    for (uint32_t s = 0; s < ns; ++s) a.split[p0 + s] = s ? 0xffffffffu : (uint32_t)b;
  }
}

// log2(o G) about the centre of the tile with origin (ox, oy), as the splat and its backward
// both evaluate it.  With (u, v) the centre minus the mean,
//   q(u + du, v + dv) = A + B du + C dv + ca du^2 + cb du dv + cc dv^2   (exact algebra);
// its float32 rounding is of the same size as that of evaluating at (u + du, v + dv)
// directly, and it costs five FMAs per texel instead of eight operations.  (sx, sy) = tile
// origin minus the mean, a double-float difference.
struct TileTaylor {
  float A, B, C, sx, sy;
};

__device__ __forceinline__ TileTaylor tile_taylor(const GRec& g, int ox, int oy) {
  TileTaylor t;
  t.sx = ((float)ox - g.mx_hi) - g.mx_lo;
  t.sy = ((float)oy - g.my_hi) - g.my_lo;
  const float uc = t.sx + 7.5f, vc = t.sy + 7.5f;
  t.A = fmaf(g.ca * uc, uc, fmaf(g.cc * vc, vc, fmaf(g.cb * uc, vc, g.l2o)));
  t.B = fmaf(2.0f * g.ca, uc, g.cb * vc);
  t.C = fmaf(g.cb, uc, 2.0f * g.cc * vc);
  return t;
}

__device__ __forceinline__ float taylor_q(float ca, float cb, float cc, float A, float B, float C, float du, float dv,
                                          float duu, float duv, float dvv) {
  return fmaf(ca, duu, fmaf(cb, duv, fmaf(cc, dvv, fmaf(B, du, fmaf(C, dv, A)))));
}

// Upper bound on log2(o G) over the texel rectangle u in [u0, u0 + 7], v in [v0, v0 + 7]
// (offsets from the mean) of the concave form q(u, v) = ca u^2 + cb u v + cc v^2 + l2o: the
// centre value if the centre lies inside, else the best point of the four edges (each a 1-D
// concave quadratic), each raised by 1e-5 of the magnitude of its terms, far above the
// float32 rounding of q at that point, so a rectangle whose texels pass the 1/255 test is
// never reported below it.  On an edge u = const the 1-D maximum lies at v = kv u, on an
// edge v = const at u = ku v (kv = -cb / (2 cc), ku = -cb / (2 ca), per Gaussian); a point
// off the exact maximum by the rounding of kv, ku lowers q by a second-order amount far
// inside the margin.
__device__ __forceinline__ float block_max_q(float ca, float cb, float cc, float l2o, float ku, float kv, float u0,
                                             float v0) {
  const float u1 = u0 + 7.0f, v1 = v0 + 7.0f;
  if (u0 <= 0.0f && 0.0f <= u1 && v0 <= 0.0f && 0.0f <= v1) return l2o;
  float best = -INFINITY;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    // e = 0, 1: edge u = u0 | u1 with v free; e = 2, 3: edge v = v0 | v1 with u free
    float u, v;
    if (e < 2) {
      u = e ? u1 : u0;
      v = fminf(fmaxf(kv * u, v0), v1);
    } else {
      v = e == 3 ? v1 : v0;
      u = fminf(fmaxf(ku * v, u0), u1);
    }
    const float tu = ca * u * u, tv = cc * v * v, tx = cb * u * v;
    const float mag = fabsf(tu) + fabsf(tv) + fabsf(tx);
    best = fmaxf(best, fmaf(1e-5f, mag, tu + tv + tx + l2o));
  }
  return best;
}

// The 8x8 quadrants of the tile (bit q = 2 qy + qx, among those of `box`) that the 1/255
// ellipse of the Gaussian reaches; (sx, sy) = tile origin minus the mean.
__device__ __forceinline__ uint32_t reached_quadrants(const GRec& g, uint32_t box, float sx, float sy) {
  // (ca, cc < 0 for every projected Gaussian: its conic is negative definite)
  const float kv = -g.cb * __builtin_amdgcn_rcpf(2.0f * g.cc), ku = -g.cb * __builtin_amdgcn_rcpf(2.0f * g.ca);
  uint32_t qm = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!((box >> q) & 1u)) continue;
    const float u0 = (float)((q & 1) << 3) + sx, v0 = (float)((q >> 1) << 3) + sy;
    if (block_max_q(g.ca, g.cb, g.cc, g.l2o, ku, kv, u0, v0) >= kLog2AlphaMin - 1e-2f) qm |= 1u << q;
  }
  return qm;
}

// LDS of one splat work item: entry e's (ca, cb, cc, A), (B, C, r, g), (b, -, -, -) with A,
// B, C the value and gradient of log2(o G) at the tile centre; per quadrant, the byte
// offsets 16 e of the entries reaching it, in order.
struct SplatLds {
  float4 p[kSegment], q[kSegment], c[kSegment];
  uint32_t list[4][kSegment];
  int cnt[4][4];                                           // [quadrant][loading wave]
};

// Where a work item's texels are: its bucket, segment, tile origin and this thread's texel.
struct SplatItem {
  int64_t bidx;
  uint32_t seg, nseg;
  int k, ox, oy, px, py;
  float du, dv;                                            // texel offset from the tile centre
};

// Stage work item `item` of a build: every thread holds one entry of the segment (its mean
// relative to the tile origin as a double-float difference, so a texel offset is one
// exact-enough add), and the work-group compacts, per 8x8 quadrant, the entries whose 1/255
// ellipse reaches it (with a margin far above the float32 error of q, so no texel is
// dropped), in order.  Returns the length of this wave's quadrant list.
__device__ __forceinline__ int splat_stage(const BuildArgs& a, uint32_t item, SplatLds& sm, SplatItem& si) {
  const uint2 it = a.items[item];
  const int64_t bidx = it.x;
  const int tile = (int)(bidx / a.K);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  si.bidx = bidx;
  si.seg = it.y;
  si.k = (int)(bidx % a.K);
  si.ox = (tile % a.ntx) << kTileShift;
  si.oy = (tile / a.ntx) << kTileShift;
  const int lxi = ((wave & 1) << 3) + (lane & 7), lyi = ((wave >> 1) << 3) + (lane >> 3);
  si.px = si.ox + lxi;
  si.py = si.oy + lyi;
  si.du = (float)lxi - 7.5f;
  si.dv = (float)lyi - 7.5f;
  const bool ok = a.hdr->overflow == 0;
  const uint32_t bb0 = a.bucket[bidx], bb1 = a.bucket[bidx + 1];
  si.nseg = seg_count(bb1 - bb0);
  const uint32_t b0 = bb0 + it.y * kSegment;
  const int n = ok ? (int)(min(bb1, b0 + kSegment) - b0) : 0;
  uint32_t qm = 0;
  if (tid < n) {
    const uint32_t ent = a.evals[b0 + tid];
    const GRec& g = a.rec[min(ent & 0x0fffffffu, (uint32_t)a.n - 1u)];
    const TileTaylor tt = tile_taylor(g, si.ox, si.oy);
    sm.p[tid] = make_float4(g.ca, g.cb, g.cc, tt.A);
    sm.q[tid] = make_float4(tt.B, tt.C, g.rgb[0], g.rgb[1]);
    sm.c[tid] = make_float4(g.rgb[2], 0.0f, 0.0f, 0.0f);
    qm = reached_quadrants(g, ent >> 28, tt.sx, tt.sy);
  }
  // waves that hold no entry (most segments are shorter than 256 entries) count zero and
  // write nothing: they skip the ranking (wave-uniform branch)
  const bool staged = wave * 64 < n;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t rank[4] = {0u, 0u, 0u, 0u};
  if (staged) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint64_t m = __ballot((qm >> q) & 1u);
      rank[q] = __popcll(m & below);
      if (lane == 0) sm.cnt[q][wave] = __popcll(m);
    }
  } else if (lane < 4) {
    sm.cnt[lane][wave] = 0;
  }
  __syncthreads();
  if (staged) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int off = 0;
      for (int w = 0; w < 4; ++w) off += w < wave ? sm.cnt[q][w] : 0;
      if ((qm >> q) & 1u) sm.list[q][off + rank[q]] = (uint32_t)tid * 16u;   // byte offset: no index math below
    }
  }
  const int my_count = sm.cnt[wave][0] + sm.cnt[wave][1] + sm.cnt[wave][2] + sm.cnt[wave][3];
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(my_count);
}

// Wave w of the 256 threads owns the 8x8 texel block at ((w & 1) * 8, (w >> 1) * 8) of the
// 16x16 tile and walks its own quadrant list, reading records from LDS (broadcast reads):
// no scalar memory traffic and no per-entry test on the critical path.
template <typename PT>
__device__ __forceinline__ void splat_item(const BuildArgs& a, uint32_t item, SplatLds& sm) {
  SplatItem si;
  const int cnt = splat_stage(a, item, sm, si);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const float du = si.du, dv = si.dv;
  const float duu = du * du, duv = du * dv, dvv = dv * dv;
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
  for (int i = 0; i < cnt; ++i) {
    const uint32_t e16 = sm.list[wave][i];
    const float4 P = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(sm.p) + e16);
    const float4 Q = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(sm.q) + e16);
    const float cb = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(sm.c) + e16)->x;
    const float4 col = make_float4(Q.z, Q.w, cb, 0.0f);
    const float q = taylor_q(P.x, P.y, P.z, P.w, Q.x, Q.y, du, dv, duu, duv, dvv);
    // excluded texels get alpha 0 (a select, not a branch)
    const float alpha = q >= kLog2AlphaMin ? fminf(kAlphaMax, __builtin_amdgcn_exp2f(q)) : 0.0f;
    const float w = alpha * T;
    C0 = fmaf(w, col.x, C0);
    C1 = fmaf(w, col.y, C1);
    C2 = fmaf(w, col.z, C2);
    T = T - w;
  }
  const int px = si.px, py = si.py;
  if (si.nseg > 1) {
    // partial (C, T) of this segment; the combine pass composes the segments in order
    const size_t slot = (size_t)a.pslot[si.bidx] + si.seg;
    a.partial[slot * (kTile * kTile) + ((py - si.oy) << kTileShift) + (px - si.ox)] = make_float4(C0, C1, C2, T);
  } else if (px < a.c.wp && py < a.c.hp) {
    store_rgba(static_cast<PT*>(a.planes), ((size_t)si.k * a.c.hp + py) * a.c.wp + px, C0, C1, C2, 1.0f - T);
  }
}

// One work-group per (tile, chunk) segment of at most kSegment entries.
template <typename PT>
__global__ __launch_bounds__(256) void splat_gs(BuildArgs a, int64_t n_buckets) {
  __shared__ SplatLds sm;
  uint32_t item;
  if (!xcd_item(blockIdx.x, a.item_start[n_buckets], a.item_shift, &item)) return;
  splat_item<PT>(a, item, sm);
}

// The splat's work, counted over the same work items and decisions: out[0] += (Gaussian,
// texel) pairs inside the plane with o G >= 1/255 (the support pairs), out[1] += (entry,
// texel) evaluations of the quadrant lists (what the splat computes), out[2] += list
// entries x 256 texels (the tile lists' superset).  out is 64 such triples, work-group b
// adding to triple b mod 64 (so the atomics do not all meet on three words); sum_slots
// adds them up.
__global__ __launch_bounds__(256) void count_splat_work(BuildArgs a, int64_t n_buckets,
                                                        unsigned long long* __restrict__ out) {
  __shared__ SplatLds sm;
  __shared__ unsigned long long part[4][2];
  uint32_t item;
  if (!xcd_item(blockIdx.x, a.item_start[n_buckets], a.item_shift, &item)) return;
  SplatItem si;
  const int cnt = splat_stage(a, item, sm, si);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const float du = si.du, dv = si.dv;
  const float duu = du * du, duv = du * dv, dvv = dv * dv;
  const bool inside = si.px < a.c.wp && si.py < a.c.hp;
  unsigned long long support = 0;
  for (int i = 0; i < cnt; ++i) {
    const uint32_t e16 = sm.list[wave][i];
    const float4 P = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(sm.p) + e16);
    const float4 Q = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(sm.q) + e16);
    const float q = taylor_q(P.x, P.y, P.z, P.w, Q.x, Q.y, du, dv, duu, duv, dvv);
    support += __popcll(__ballot(inside && q >= kLog2AlphaMin));
  }
  if (lane == 0) {
    part[wave][0] = support;
    part[wave][1] = (unsigned long long)cnt * 64u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t bb0 = a.bucket[si.bidx], bb1 = a.bucket[si.bidx + 1];
    const uint32_t b0 = bb0 + si.seg * kSegment;
    const unsigned long long n = a.hdr->overflow == 0 ? min(bb1, b0 + kSegment) - b0 : 0u;
    unsigned long long* o = out + 3 * (blockIdx.x & 63u);
    atomicAdd(&o[0], part[0][0] + part[1][0] + part[2][0] + part[3][0]);
    atomicAdd(&o[1], part[0][1] + part[1][1] + part[2][1] + part[3][1]);
    atomicAdd(&o[2], n * (unsigned long long)(kTile * kTile));
  }
}

__global__ void sum_slots(const unsigned long long* __restrict__ slots, unsigned long long* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= 3) return;
  unsigned long long t = 0;
  for (int i = 0; i < 64; ++i) t += slots[3 * i + c];
  out[c] = t;
}

// ---------------------------------------------------------------------------------------
// SH splat (the spherical-harmonic planes of Fig. 6): the texels blend the Gaussians'
// NC x 3 colour coefficients with the weights alpha T of the RGB splat, in the same Taylor
// form and with the same per-quadrant lists.  One work-group per (tile, chunk) bucket walks
// the bucket's entries in order, kShSplatSeg at a time, so its transmittance carries over
// and no partial tiles are needed (a texel's state is 3 NC + 1 floats).  Per step, thread t
// stages entry t's quadratic form and Gaussian index in LDS, the work-group compacts the
// entries reaching each quadrant (stable), and each wave walks its quadrant's list.  A wave's entry is uniform, so its coefficients come through scalar
// loads (read-only data, constant address space) and feed the blend FMAs as scalar
// operands: no LDS traffic and no vector registers for them.  The texel is stored as q_0
// (r, g, b), A, q_1 .. q_{NC-1} (r, g, b), zero padding.
// ---------------------------------------------------------------------------------------
constexpr int kShSplatSeg = 256;
typedef const float __attribute__((address_space(4))) ConstF32;

template <int NC>
__global__ __launch_bounds__(256) void splat_sh_gs(BuildArgs a, int64_t n_buckets) {
  constexpr int NF = 3 * NC;                     // coefficient floats per Gaussian
  constexpr int TF = sh_texel_floats(NC);
  __shared__ float4 s_p[kShSplatSeg];            // (ca, cb, cc, A)
  __shared__ float2 s_q[kShSplatSeg];            // (B, C)
  __shared__ uint32_t s_gi[kShSplatSeg];
  __shared__ uint8_t s_list[4][kShSplatSeg];
  __shared__ int s_cnt[4][4];                    // [quadrant][loading wave]
  const int64_t bidx = blockIdx.x;
  if (bidx >= n_buckets) return;
  const int tile = (int)(bidx / a.K), k = (int)(bidx % a.K);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ox = (tile % a.ntx) << kTileShift, oy = (tile / a.ntx) << kTileShift;
  const int lxi = ((wave & 1) << 3) + (lane & 7), lyi = ((wave >> 1) << 3) + (lane >> 3);
  const int px = ox + lxi, py = oy + lyi;
  const float du = (float)lxi - 7.5f, dv = (float)lyi - 7.5f;
  const float duu = du * du, duv = du * dv, dvv = dv * dv;
  const bool ok = a.hdr->overflow == 0;
  const uint32_t bb0 = a.bucket[bidx], bb1 = ok ? a.bucket[bidx + 1] : bb0;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  ConstF32* sh = (ConstF32*)a.sh;
  float acc[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) acc[j] = 0.0f;
  float T = 1.0f;
  for (uint32_t b0 = bb0; b0 < bb1; b0 += kShSplatSeg) {
    const int n = (int)min(bb1 - b0, (uint32_t)kShSplatSeg);
    __syncthreads();                             // the previous step is consumed
    uint32_t qm = 0;
    if (tid < n) {
      const uint32_t ent = a.evals[b0 + tid];
      const uint32_t gi = min(ent & 0x0fffffffu, (uint32_t)a.n - 1u);
      const GRec& g = a.rec[gi];
      const TileTaylor tt = tile_taylor(g, ox, oy);
      s_p[tid] = make_float4(g.ca, g.cb, g.cc, tt.A);
      s_q[tid] = make_float2(tt.B, tt.C);
      s_gi[tid] = gi;
      qm = reached_quadrants(g, ent >> 28, tt.sx, tt.sy);
    }
    uint32_t rank[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint64_t m = __ballot((qm >> q) & 1u);
      rank[q] = __popcll(m & below);
      if (lane == 0) s_cnt[q][wave] = __popcll(m);
    }
    __syncthreads();
    int my_count = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int off = 0;
      for (int w = 0; w < 4; ++w) off += w < wave ? s_cnt[q][w] : 0;
      if ((qm >> q) & 1u) s_list[q][off + rank[q]] = (uint8_t)tid;
      if (q == wave) my_count = s_cnt[q][0] + s_cnt[q][1] + s_cnt[q][2] + s_cnt[q][3];
    }
    __syncthreads();
    const int cnt = __builtin_amdgcn_readfirstlane(my_count);
    for (int i = 0; i < cnt; ++i) {
      const int e = __builtin_amdgcn_readfirstlane(s_list[wave][i]);
      const uint32_t gi = __builtin_amdgcn_readfirstlane(s_gi[e]);
      ConstF32* c = sh + (size_t)gi * NF;
      const float4 P = s_p[e];
      const float2 Q = s_q[e];
      const float q = taylor_q(P.x, P.y, P.z, P.w, Q.x, Q.y, du, dv, duu, duv, dvv);
      const float alpha = q >= kLog2AlphaMin ? fminf(kAlphaMax, __builtin_amdgcn_exp2f(q)) : 0.0f;
      const float w = alpha * T;
#pragma unroll
      for (int j = 0; j < NF; ++j) acc[j] = fmaf(w, c[j], acc[j]);
      T = T - w;
    }
  }
  if (px < a.c.wp && py < a.c.hp) {
    float t[TF];
    t[0] = acc[0];
    t[1] = acc[1];
    t[2] = acc[2];
    t[3] = 1.0f - T;
#pragma unroll
    for (int j = 3; j < NF; ++j) t[j + 1] = acc[j];
#pragma unroll
    for (int j = NF + 1; j < TF; ++j) t[j] = 0.0f;
    float4* dst = reinterpret_cast<float4*>(static_cast<float*>(a.planes) + (((size_t)k * a.c.hp + py) * a.c.wp + px) * TF);
#pragma unroll
    for (int j = 0; j < TF / 4; ++j) dst[j] = make_float4(t[4 * j], t[4 * j + 1], t[4 * j + 2], t[4 * j + 3]);
  }
}

template <typename PT>
__device__ void combine_bucket(const BuildArgs& a, int64_t bidx) {
  const uint32_t nseg = seg_count(a.bucket[bidx + 1] - a.bucket[bidx]);
  const int tile = (int)(bidx / a.K), k = (int)(bidx % a.K);
  const int ox = (tile % a.ntx) << kTileShift, oy = (tile / a.ntx) << kTileShift;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = ox + ((wave & 1) << 3) + (lane & 7), py = oy + ((wave >> 1) << 3) + (lane >> 3);
  const float4* p = a.partial + (size_t)a.pslot[bidx] * (kTile * kTile) + ((py - oy) << kTileShift) + (px - ox);
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
  for (uint32_t s0 = 0; s0 < nseg; s0 += 4) {
    float4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)                            // the loads in flight together
      v[q] = s0 + q < nseg ? p[(size_t)(s0 + q) * (kTile * kTile)] : make_float4(0.f, 0.f, 0.f, 1.f);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (s0 + q >= nseg) break;
      C0 = fmaf(T, v[q].x, C0);
      C1 = fmaf(T, v[q].y, C1);
      C2 = fmaf(T, v[q].z, C2);
      T = T * v[q].w;
    }
  }
  if (px < a.c.wp && py < a.c.hp)
    store_rgba(static_cast<PT*>(a.planes), ((size_t)k * a.c.hp + py) * a.c.wp + px, C0, C1, C2, 1.0f - T);
}

// Over-composite the segments of every split bucket: work-groups stride over the partial
// slots, and the first slot of each split bucket takes that bucket.
template <typename PT>
__global__ __launch_bounds__(256) void combine_segments(BuildArgs a, int64_t n_buckets) {
  const uint32_t nslots = a.pslot[n_buckets];
  for (uint32_t i = blockIdx.x; i < nslots; i += gridDim.x) {
    const uint32_t b = a.split[i];
    if (b != 0xffffffffu) combine_bucket<PT>(a, b);
  }
}

// The splat and merge of several builds in one launch each: the work items of builds
// [0 .. n) form one list, build after build, and so do their partial slots.  A one-thread
// kernel first writes the prefix sums of the builds' counts (read on the device, after the
// builds' lists): prefix[0 .. n] of the items, prefix[n + 1 .. 2n + 1] of the partial
// slots.  A work-group finds its build by a scan of that short array.  Items are dealt to
// the XCDs as in splat_gs.
__global__ void jobs_prefix(const BuildArgs* __restrict__ args, SplatJobs jobs) {
  uint32_t* p = jobs.prefix;
  uint32_t t = 0, u = 0;
  p[0] = 0;
  p[jobs.n + 1] = 0;
  for (int j = 0; j < jobs.n; ++j) {
    t += args[j].item_start[jobs.n_buckets[j]];
    u += args[j].pslot[jobs.n_buckets[j]];
    p[j + 1] = t;
    p[jobs.n + 2 + j] = u;
  }
}

__device__ __forceinline__ int job_of(const uint32_t* __restrict__ prefix, int n, uint32_t w, uint32_t* local) {
  int j = 0;
  while (j + 1 < n && w >= prefix[j + 1]) ++j;
  *local = w - prefix[j];
  return j;
}

template <typename PT>
__global__ __launch_bounds__(256) void splat_gs_jobs(const BuildArgs* __restrict__ args, SplatJobs jobs) {
  __shared__ SplatLds sm;
  uint32_t w, item;
  if (!xcd_item(blockIdx.x, jobs.prefix[jobs.n], jobs.item_shift, &w)) return;
  const int j = job_of(jobs.prefix, jobs.n, w, &item);
  splat_item<PT>(args[j], item, sm);
}

template <typename PT>
__global__ __launch_bounds__(256) void combine_jobs(const BuildArgs* __restrict__ args, SplatJobs jobs) {
  const uint32_t* pp = jobs.prefix + jobs.n + 1;
  const uint32_t nslots = pp[jobs.n];
  for (uint32_t i = blockIdx.x; i < nslots; i += gridDim.x) {
    uint32_t slot;
    const int j = job_of(pp, jobs.n, i, &slot);
    const uint32_t b = args[j].split[slot];
    if (b != 0xffffffffu) combine_bucket<PT>(args[j], b);
  }
}

// ---------------------------------------------------------------------------------------
// Backward of the splat.  Per texel of a bucket with cotangents gC = dL/dC, gA = dL/dA of
// its plane texel, over the bucket's Gaussians i (front to back, alpha_i, colour c_i):
//   dL/dc_i     = T_i alpha_i gC
//   dL/dalpha_i = T_i (gC . (c_i - R_{i+1}) + gA S_{i+1}),
//   R_i = alpha_i c_i + (1 - alpha_i) R_{i+1},  S_i = (1 - alpha_i) S_{i+1},
// with R, S of the bucket's end = (0, 1), evaluated back to front.  A work item is one
// segment of a bucket: its T at the segment start and (R, S) at its end come from the
// other segments' forward partials (C_s, T_s).  Inside the segment T_i is recomputed: a
// forward sweep stores T every 16 entries (LDS), then each block of 16 is swept forward
// again into registers and walked backwards.  alpha = min(0.99, 2^q), q = l2o + ca dx^2 +
// cb dx dy + cc dy^2 (evaluated in the forward's Taylor form, so both take the same
// decisions), included iff q >= log2(1/255): d alpha/dq = alpha ln 2 where included and not
// clamped.  The segment's Gaussians are staged in LDS once.  Each wave reduces its 64
// texels' contributions per Gaussian and adds them to the Gaussian's accumulators.
// ---------------------------------------------------------------------------------------
constexpr float kLn2 = 0.69314718055994531f;
constexpr int kBwdBlock = 16;

// Sum of v over the wave, complete in lane 63 (the other lanes hold partial sums): inclusive
// sums within each row of 16 lanes (data-parallel-primitive shifts by 1, 2, 4, 8; lanes
// shifted in from outside the row add zero), then row 0's total added to row 1 and row 2's
// to row 3 (broadcast of lane 15), then lane 31's to rows 2 and 3 (broadcast of lane 31).
// VALU only, where a butterfly of lane shuffles goes through the LDS crossbar.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, kRowMask, 0xf, true));
}
__device__ __forceinline__ float wave_sum_last(float v) {
  v = dpp_add<0x111, 0xf>(v);                              // row_shr:1
  v = dpp_add<0x112, 0xf>(v);                              // row_shr:2
  v = dpp_add<0x114, 0xf>(v);                              // row_shr:4
  v = dpp_add<0x118, 0xf>(v);                              // row_shr:8
  v = dpp_add<0x142, 0xa>(v);                              // row_bcast:15 into rows 1, 3
  v = dpp_add<0x143, 0xc>(v);                              // row_bcast:31 into rows 2, 3
  return v;
}

__global__ __launch_bounds__(256) void splat_bwd_gs(BuildArgs a, int64_t n_buckets) {
  __shared__ float ckpt[kSegment / kBwdBlock][256];
  // entry e of the segment, staged once: (ca, cb, cc, A), (B, C, r, g), (b, sx, sy, entry
  // bits: Gaussian index and quadrant mask); the same Taylor form the forward evaluated
  __shared__ float4 s_p[kSegment], s_q[kSegment], s_c[kSegment];
  uint32_t item;
  if (!xcd_item(blockIdx.x, a.item_start[n_buckets], a.item_shift, &item)) return;
  if (a.hdr->overflow) return;
  const uint2 it = a.items[item];
  const int64_t bidx = it.x;
  const int tile = (int)(bidx / a.K), k = (int)(bidx % a.K);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ox = (tile % a.ntx) << kTileShift, oy = (tile / a.ntx) << kTileShift;
  const int lxi = ((wave & 1) << 3) + (lane & 7), lyi = ((wave >> 1) << 3) + (lane >> 3);
  const int px = ox + lxi, py = oy + lyi;
  const float lx = (float)lxi, ly = (float)lyi;
  const float du = lx - 7.5f, dv = ly - 7.5f;
  const float duu = du * du, duv = du * dv, dvv = dv * dv;
  const uint32_t* __restrict__ ev = a.evals;
  const uint32_t bb0 = a.bucket[bidx], bb1 = a.bucket[bidx + 1];
  const uint32_t nseg = seg_count(bb1 - bb0);
  const uint32_t b0 = bb0 + it.y * kSegment, b1 = min(bb1, b0 + kSegment);
  const int n = (int)(b1 - b0);
  if (tid < n) {
    const uint32_t ent = ev[b0 + tid];
    const uint32_t idx = min(ent & 0x0fffffffu, (uint32_t)a.n - 1u);
    const GRec& g = a.rec[idx];
    const TileTaylor tt = tile_taylor(g, ox, oy);
    s_p[tid] = make_float4(g.ca, g.cb, g.cc, tt.A);
    s_q[tid] = make_float4(tt.B, tt.C, g.rgb[0], g.rgb[1]);
    // the quadrants the forward evaluated
    const uint32_t qm = reached_quadrants(g, ent >> 28, tt.sx, tt.sy) << 28;
    s_c[tid] = make_float4(g.rgb[2], tt.sx, tt.sy, __uint_as_float(idx | qm));
  }
  const bool in_plane = px < a.c.wp && py < a.c.hp;
  float4 gp = make_float4(0.f, 0.f, 0.f, 0.f);
  if (in_plane) gp = reinterpret_cast<const float4*>(a.d_planes)[((size_t)k * a.c.hp + py) * a.c.wp + px];
  // transmittance in front of the segment, colour and transmittance behind it
  float Tin = 1.0f, Rr = 0.f, Rg = 0.f, Rb = 0.f, Sf = 1.0f;
  if (nseg > 1) {
    const float4* part = a.partial + (size_t)a.pslot[bidx] * (kTile * kTile) + ((py - oy) << kTileShift) + (px - ox);
    for (uint32_t s = 0; s < it.y; ++s) Tin *= part[(size_t)s * (kTile * kTile)].w;
    for (uint32_t s = nseg - 1; s > it.y; --s) {
      const float4 p = part[(size_t)s * (kTile * kTile)];
      Rr = fmaf(p.w, Rr, p.x);
      Rg = fmaf(p.w, Rg, p.y);
      Rb = fmaf(p.w, Rb, p.z);
      Sf *= p.w;
    }
  }
  __syncthreads();
  const uint32_t qbit = 1u << (28 + wave);
  // entry bits (uniform over the work-group)
  auto bits_of = [&](int e) { return __builtin_amdgcn_readfirstlane(__float_as_uint(s_c[e].w)); };
  auto q_of = [&](int e) {
    const float4 P = s_p[e];
    const float4 Q = s_q[e];
    return taylor_q(P.x, P.y, P.z, P.w, Q.x, Q.y, du, dv, duu, duv, dvv);
  };
  auto alpha_of = [](float q) { return q >= kLog2AlphaMin ? fminf(kAlphaMax, __builtin_amdgcn_exp2f(q)) : 0.0f; };
  // forward sweep: T (within the segment) at the start of every block of kBwdBlock entries
  float T = 1.0f;
  for (int e = 0; e < n; ++e) {
    if ((e & (kBwdBlock - 1)) == 0) ckpt[e / kBwdBlock][tid] = T;
    if (!(bits_of(e) & qbit)) continue;
    T = T - alpha_of(q_of(e)) * T;
  }
  const int nblk = (n + kBwdBlock - 1) / kBwdBlock;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int e0 = blk * kBwdBlock;
    float Tv[kBwdBlock];
    float Tb = ckpt[blk][tid];
#pragma unroll
    for (int j = 0; j < kBwdBlock; ++j) {
      Tv[j] = Tb;
      const int e = e0 + j;
      if (e < n && (bits_of(e) & qbit)) Tb = Tb - alpha_of(q_of(e)) * Tb;
    }
#pragma unroll
    for (int j = kBwdBlock - 1; j >= 0; --j) {
      const int e = e0 + j;
      if (e >= n) continue;
      const uint32_t bits = bits_of(e);
      if (!(bits & qbit)) continue;                         // the Gaussian misses this quadrant
      const uint32_t idx = bits & 0x0fffffffu;
      const float4 P = s_p[e];
      const float4 Q = s_q[e];
      const float4 Cc = s_c[e];
      const float ca = P.x, cb = P.y, cc = P.z;
      const float cr = Q.z, cg = Q.w, cbl = Cc.x;
      const float q = taylor_q(ca, cb, cc, P.w, Q.x, Q.y, du, dv, duu, duv, dvv);
      const float alpha = alpha_of(q);
      const float dx = lx + Cc.y, dy = ly + Cc.z;           // texel minus the mean
      const float W = Tin * Tv[j];
      const float gal = W * ((gp.x * (cr - Rr) + gp.y * (cg - Rg) + gp.z * (cbl - Rb)) + gp.w * Sf);
      const float wa = W * alpha;
      const float om = 1.0f - alpha;
      Rr = fmaf(om, Rr, alpha * cr);
      Rg = fmaf(om, Rg, alpha * cg);
      Rb = fmaf(om, Rb, alpha * cbl);
      Sf = om * Sf;
      const bool smooth = q >= kLog2AlphaMin && __builtin_amdgcn_exp2f(q) < kAlphaMax;
      const float gq = smooth ? gal * alpha * kLn2 : 0.0f;
      float v[kGradSlots];
      v[0] = gq * dx * dx;
      v[1] = gq * dx * dy;
      v[2] = gq * dy * dy;
      v[3] = -gq * fmaf(2.0f * ca, dx, cb * dy);
      v[4] = -gq * fmaf(2.0f * cc, dy, cb * dx);
      v[5] = gq;
      v[6] = wa * gp.x;
      v[7] = wa * gp.y;
      v[8] = wa * gp.z;
      // the wave's sums, read out of lane 63 as wave-uniform values, added by lane 0
      float t[kGradSlots];
#pragma unroll
      for (int s = 0; s < kGradSlots; ++s)
        t[s] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_last(v[s])), 63));
      if (lane == 0) {
        float* dst = a.ggrad + (size_t)idx * kGradSlots;
#pragma unroll
        for (int s = 0; s < kGradSlots; ++s)
          if (t[s] != 0.0f) atomicAdd(dst + s, t[s]);
      }
    }
  }
}

// Chain rule of the projection (preprocess_gs, in reverse), one thread per Gaussian.
// Accumulators -> conic (ca, cb, cc) -> Sigma'^-1 -> Sigma' = (J M)(J M)^T + f' I with
// M = W R(q) diag(e^l) -> J (camera-space mean), M -> (R(q), e^l) -> quaternion (through
// its normalisation) and log-scales; projected mean -> camera-space mean -> means; log2 o
// -> opacity.
__global__ __launch_bounds__(256) void preprocess_bwd_gs(BuildArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Consts& c = a.c;
  float gm[3] = {0.f, 0.f, 0.f}, gl[3] = {0.f, 0.f, 0.f}, gqt[4] = {0.f, 0.f, 0.f, 0.f}, go = 0.f, gc[3] = {0.f, 0.f, 0.f};
  const float mx = a.means[3 * i], my = a.means[3 * i + 1], mz = a.means[3 * i + 2];
  const KeyCull kc = key_and_cull(c, mx, my, mz);
  if (kc.vis) {
    const float* acc = a.ggrad + (size_t)i * kGradSlots;
    const float g_ca = acc[0], g_cb = acc[1], g_cc = acc[2], g_mux = acc[3], g_muy = acc[4], g_l2o = acc[5];
    gc[0] = acc[6];
    gc[1] = acc[7];
    gc[2] = acc[8];
    // forward quantities (float32, as preprocess_gs)
    float qw = a.quats[4 * i], qx = a.quats[4 * i + 1], qy = a.quats[4 * i + 2], qz = a.quats[4 * i + 3];
    const float qnorm = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    const float qn = 1.0f / qnorm;
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    const float Rg[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                         2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                         2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
    const float s[3] = {expf(a.log_scales[3 * i]), expf(a.log_scales[3 * i + 1]), expf(a.log_scales[3 * i + 2])};
    float M[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k)
        M[3 * r + k] = (c.R[3 * r] * Rg[k] + c.R[3 * r + 1] * Rg[3 + k] + c.R[3 * r + 2] * Rg[6 + k]) * s[k];
    const float x = kc.xc, y = kc.yc, z = kc.key - c.d_fwd;
    const float iz = 1.0f / z;
    const float j00 = c.fpx * iz, j02 = -c.fpx * x * iz * iz, j11 = c.fpy * iz, j12 = -c.fpy * y * iz * iz;
    float u[3], v[3];
    for (int k = 0; k < 3; ++k) {
      u[k] = j00 * M[k] + j02 * M[6 + k];
      v[k] = j11 * M[3 + k] + j12 * M[6 + k];
    }
    const float sa = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + c.f_dil;
    const float sb = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    const float sc = (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) + c.f_dil;
    const float bb = sb * sb;
    const float det = fmaxf(fmaf(sa, sc, -bb) + fmaf(-sb, sb, bb), fmaxf(c.f_dil * c.f_dil, 1e-10f));
    const float idet = 1.0f / det;
    // conic = -1/2 log2e Sigma'^-1 with cb carrying both off-diagonal entries
    const float h = 0.5f * kLog2e;
    const float G00 = -h * g_ca, G01 = -h * g_cb, G11 = -h * g_cc;     // dL/d(Sigma'^-1) per entry
    const float I00 = sc * idet, I01 = -sb * idet, I11 = sa * idet;
    const float m00 = G00 * I00 + G01 * I01, m01 = G00 * I01 + G01 * I11;
    const float m10 = G01 * I00 + G11 * I01, m11 = G01 * I01 + G11 * I11;
    const float S00 = -(I00 * m00 + I01 * m10), S11 = -(I01 * m01 + I11 * m11);
    const float S01 = -0.5f * ((I00 * m01 + I01 * m11) + (I01 * m00 + I11 * m10));
    // Sigma' = U U^T + f' I, U rows u, v:  dL/dU = 2 S U
    float gu[3], gv[3];
    for (int k = 0; k < 3; ++k) {
      gu[k] = 2.0f * (S00 * u[k] + S01 * v[k]);
      gv[k] = 2.0f * (S01 * u[k] + S11 * v[k]);
    }
    // U = J M
    float gM[9];
    float g_j00 = 0.f, g_j02 = 0.f, g_j11 = 0.f, g_j12 = 0.f;
    for (int k = 0; k < 3; ++k) {
      gM[k] = gu[k] * j00;
      gM[3 + k] = gv[k] * j11;
      gM[6 + k] = gu[k] * j02 + gv[k] * j12;
      g_j00 += gu[k] * M[k];
      g_j02 += gu[k] * M[6 + k];
      g_j11 += gv[k] * M[3 + k];
      g_j12 += gv[k] * M[6 + k];
    }
    // J and the projected mean as functions of the camera-space mean (x, y, z)
    const float iz2 = iz * iz, iz3 = iz2 * iz;
    const float g_x = g_j02 * (-c.fpx * iz2) + g_mux * c.fpx * iz;
    const float g_y = g_j12 * (-c.fpy * iz2) + g_muy * c.fpy * iz;
    const float g_z = g_j00 * (-c.fpx * iz2) + g_j02 * (2.0f * c.fpx * x * iz3) + g_j11 * (-c.fpy * iz2) +
                      g_j12 * (2.0f * c.fpy * y * iz3) - g_mux * c.fpx * x * iz2 - g_muy * c.fpy * y * iz2;
    for (int j = 0; j < 3; ++j) gm[j] = c.R[j] * g_x + c.R[3 + j] * g_y + c.R[6 + j] * g_z;
    // M = W R diag(s):  dL/dl_k = sum_r gM[r][k] M[r][k];  dL/dR[j][k] = s_k sum_r W[r][j] gM[r][k]
    float gR[9];
    for (int k = 0; k < 3; ++k) {
      gl[k] = gM[k] * M[k] + gM[3 + k] * M[3 + k] + gM[6 + k] * M[6 + k];
      for (int j = 0; j < 3; ++j)
        gR[3 * j + k] = s[k] * (c.R[j] * gM[k] + c.R[3 + j] * gM[3 + k] + c.R[6 + j] * gM[6 + k]);
    }
    // rotation of the normalised quaternion (w, x, y, z)
    const float gw = 2.f * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
    const float gx = 2.f * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.f * qx * gR[4] - qw * gR[5] + qz * gR[6] +
                            qw * gR[7] - 2.f * qx * gR[8]);
    const float gy = 2.f * (-2.f * qy * gR[0] + qx * gR[1] + qw * gR[2] + qx * gR[3] + qz * gR[5] - qw * gR[6] +
                            qz * gR[7] - 2.f * qy * gR[8]);
    const float gz = 2.f * (-2.f * qz * gR[0] - qw * gR[1] + qx * gR[2] + qw * gR[3] - 2.f * qz * gR[4] +
                            qy * gR[5] + qx * gR[6] + qy * gR[7]);
    const float dot = gw * qw + gx * qx + gy * qy + gz * qz;
    gqt[0] = (gw - qw * dot) * qn;
    gqt[1] = (gx - qx * dot) * qn;
    gqt[2] = (gy - qy * dot) * qn;
    gqt[3] = (gz - qz * dot) * qn;
    go = g_l2o / (a.opacity[i] * kLn2);
  }
  for (int j = 0; j < 3; ++j) {
    a.grads.means[3 * i + j] = gm[j];
    a.grads.log_scales[3 * i + j] = gl[j];
    a.grads.rgb[3 * i + j] = gc[j];
  }
  for (int j = 0; j < 4; ++j) a.grads.quats[4 * i + j] = gqt[j];
  a.grads.opacity[i] = go;
}

// Copy of the tile lists for inspection: bucket starts widened to int64, entries reduced to
// their primitive index (the quadrant mask of bits 28..31 dropped).
__global__ __launch_bounds__(256) void copy_tile_lists(const uint32_t* bucket, const uint32_t* evals, int64_t n_buckets,
                                                      int64_t* bucket_out, int32_t* entries_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (bucket_out && i <= n_buckets) bucket_out[i] = bucket[i];
  if (entries_out && i < (int64_t)bucket[n_buckets]) entries_out[i] = (int32_t)(evals[i] & 0x0fffffffu);
}

__global__ void write_table(float* dst, TableChunk t) {
  const int i = threadIdx.x;
  if (i < t.count) dst[t.offset + i] = t.v[i];
}

}  // namespace

hipError_t upload_table(float* dst, const float* host, int n, hipStream_t s) {
  for (int off = 0; off < n; off += kTableChunk) {
    TableChunk t;
    t.offset = off;
    t.count = n - off < kTableChunk ? n - off : kTableChunk;
    for (int i = 0; i < t.count; ++i) t.v[i] = host[off + i];
    hipLaunchKernelGGL(write_table, dim3(1), dim3(kTableChunk), 0, s, dst, t);
  }
  return hipGetLastError();
}

hipError_t tile_lists_launch(const BuildArgs& a, const BuildLayout& L, int64_t* bucket_start, int32_t* entries,
                             hipStream_t s) {
  const int64_t n = std::max<int64_t>(L.n_buckets + 1, L.cap);
  hipLaunchKernelGGL(copy_tile_lists, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a.bucket, a.evals,
                     L.n_buckets, bucket_start, entries);
  return hipGetLastError();
}

// Digit width of the entry sort by tile (LF_TILE_DIGIT_BITS overrides, 4..11).
int tile_digit_bits() {
  if (const char* e = getenv("LF_TILE_DIGIT_BITS")) {
    const int b = atoi(e);
    if (b >= 4 && b <= 11) return b;
  }
  return kTileDigitBits;
}

// Digit width of the depth-key sort (LF_KEY_DIGIT_BITS overrides, 4..11).
int key_digit_bits() {
  if (const char* e = getenv("LF_KEY_DIGIT_BITS")) {
    const int b = atoi(e);
    if (b >= 4 && b <= 11) return b;
  }
  return kKeyDigitBits;
}

// The splat's work items in the chosen order: segment counts, their scan (item starts; and
// the partial-tile slots, whose values do not depend on the order) and the items.  The
// items scan state must be zero on entry.
hipError_t emit_work_items(BuildArgs& a, const BuildLayout& L, hipStream_t s, int chunk_major) {
  const unsigned gB = (unsigned)((L.n_buckets + 255) / 256);
  hipLaunchKernelGGL(bucket_segments, dim3(gB), dim3(256), 0, s, a, L.n_buckets, chunk_major);
  hipError_t e = exclusive_scan_pair_u32(a.nseg, a.item_start, a.pcnt, a.pslot, L.n_buckets, a.scan_state_items,
                                         &a.hdr->stalled, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(emit_items, dim3(gB), dim3(256), 0, s, a, L.n_buckets, chunk_major);
  return hipGetLastError();
}

hipError_t build_lists(BuildArgs& a, const BuildLayout& L, hipStream_t s, Profiler* prof, bool* done) {
  hipError_t e;
  *done = false;
  const unsigned gN = (unsigned)((a.n + 255) / 256);
  {
    PhaseScope ps(prof, LF_PHASE_PREPROCESS, s);
    // counters, digit totals of both sorts and the scan states start at zero
    if ((e = fill(reinterpret_cast<uint32_t*>(a.hdr), a.clear_words, 0u, s)) != hipSuccess) return e;
    if (a.n == 0) {
      // nothing to rasterise: transparent planes at D_focal (or the inverse-depth table)
      const int texel_words = a.sh_coef ? sh_texel_floats(a.sh_coef)
                              : a.plane_dtype == LF_F32 ? 4 : a.plane_dtype == LF_U8 ? 1 : 2;
      const size_t words = (size_t)a.K * a.c.hp * a.c.wp * texel_words;
      if ((e = fill(reinterpret_cast<uint32_t*>(a.planes), (int64_t)words, 0u, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(chunk_table, dim3(1), dim3(1024), 0, s, a, a.keys);
      *done = true;
      return hipGetLastError();
    }
    if (a.kind == LF_VOXELS) {
      if ((e = launch_preprocess_vox(a, s)) != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL(preprocess_gs, dim3(gN), dim3(256), 0, s, a);
    }
  }
  // (key, index) order
  int alt = 0;
  {
    PhaseScope ps(prof, LF_PHASE_SORT, s);
    if ((e = radix_sort_pairs(a.keys, a.vals, a.keys_alt, a.vals_alt, a.n, nullptr, 0, 32, a.radix_tmp, a.ghist_key,
                              &a.hdr->stalled, &alt, s, key_digit_bits())) != hipSuccess)
      return e;
  }
  const uint32_t* skeys = alt ? a.keys_alt : a.keys;
  const uint32_t* svals = alt ? a.vals_alt : a.vals;
  {
    PhaseScope ps(prof, LF_PHASE_BIN, s);
    hipLaunchKernelGGL(find_nvis, dim3(gN), dim3(256), 0, s, a, skeys);
    hipLaunchKernelGGL(rank_pass, dim3(gN), dim3(256), 0, s, a, skeys, svals);
    hipLaunchKernelGGL(chunk_table, dim3(1), dim3(1024), 0, s, a, skeys);
    if ((e = exclusive_scan_u64(a.ntiles_r, a.offsets, a.n, a.scan_state_offsets, &a.hdr->stalled, s, a.heads,
                                a.n_heads, 8)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(emit_entries, dim3((unsigned)((a.capacity + 255) / 256)), dim3(256), 0, s, a, svals);
    // stable sort of the entries by tile (entries beyond the capacity are never read)
    int ealt = 0;
    if ((e = radix_sort_pairs(a.ekeys, a.evals, a.ekeys_alt, a.evals_alt, a.capacity,
                              reinterpret_cast<const int64_t*>(&a.hdr->entries), L.chunk_bits, L.tile_bits,
                              a.radix_tmp, a.ghist_tile, &a.hdr->stalled, &ealt, s, tile_digit_bits())) != hipSuccess)
      return e;
    if (ealt) a.evals = a.evals_alt;
    const uint32_t* sekeys = ealt ? a.ekeys_alt : a.ekeys;
    hipLaunchKernelGGL(bucket_bounds, dim3((unsigned)((L.n_buckets + 1 + 255) / 256)), dim3(256), 0, s, a, sekeys,
                       L.n_buckets);
    // work items: buckets split into segments of at most kSegment entries (chunk-major for
    // the Gaussian splat, whose records then stay in one XCD's L2; the voxel splat, which
    // reads its records with scalar loads, ran in 0.26 ms tile-major against 0.36 ms
    // chunk-major on a 335k-voxel frame)
    if ((e = emit_work_items(a, L, s, a.kind == LF_GAUSSIANS)) != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t build_splat(BuildArgs& a, const BuildLayout& L, hipStream_t s, Profiler* prof) {
  hipError_t e;
  if (a.sh_coef) {
    // SH planes: one work-group per bucket, no partial tiles to merge
    PhaseScope ps(prof, LF_PHASE_SPLAT, s);
    const dim3 grid((unsigned)L.n_buckets);
    switch (a.sh_coef) {
      case 1: hipLaunchKernelGGL((splat_sh_gs<1>), grid, dim3(256), 0, s, a, L.n_buckets); break;
      case 4: hipLaunchKernelGGL((splat_sh_gs<4>), grid, dim3(256), 0, s, a, L.n_buckets); break;
      case 9: hipLaunchKernelGGL((splat_sh_gs<9>), grid, dim3(256), 0, s, a, L.n_buckets); break;
      default: hipLaunchKernelGGL((splat_sh_gs<16>), grid, dim3(256), 0, s, a, L.n_buckets); break;
    }
    return hipGetLastError();
  }
  // voxel planes are splatted in float32 into the workspace's stage; the low-pass then
  // stores each plane once in its own dtype (one rounding of the filtered value)
  void* const planes_out = a.planes;
  const int32_t dtype_out = a.plane_dtype;
  if (a.kind == LF_VOXELS) {
    a.planes = a.stage;
    a.plane_dtype = LF_F32;
  }
  {
    PhaseScope ps(prof, LF_PHASE_SPLAT, s);
    const dim3 grid((unsigned)xcd_grid(L.max_items, a.item_shift));
    if (a.kind == LF_VOXELS) {
      if ((e = launch_splat_vox(a, L, s)) != hipSuccess) return e;
    } else switch (a.plane_dtype) {
      case LF_F16: hipLaunchKernelGGL((splat_gs<__half>), grid, dim3(256), 0, s, a, L.n_buckets); break;
      case LF_BF16: hipLaunchKernelGGL((splat_gs<__hip_bfloat16>), grid, dim3(256), 0, s, a, L.n_buckets); break;
      case LF_U8: hipLaunchKernelGGL((splat_gs<uint8_t>), grid, dim3(256), 0, s, a, L.n_buckets); break;
      default: hipLaunchKernelGGL((splat_gs<float>), grid, dim3(256), 0, s, a, L.n_buckets); break;
    }
  }
  {
    PhaseScope ps(prof, LF_PHASE_MERGE, s);
    const dim3 grid((unsigned)std::min<int64_t>(L.max_partial, kCombineGroups));
    switch (a.plane_dtype) {
      case LF_F16: hipLaunchKernelGGL((combine_segments<__half>), grid, dim3(256), 0, s, a, L.n_buckets); break;
      case LF_BF16: hipLaunchKernelGGL((combine_segments<__hip_bfloat16>), grid, dim3(256), 0, s, a, L.n_buckets); break;
      case LF_U8: hipLaunchKernelGGL((combine_segments<uint8_t>), grid, dim3(256), 0, s, a, L.n_buckets); break;
      default: hipLaunchKernelGGL((combine_segments<float>), grid, dim3(256), 0, s, a, L.n_buckets); break;
    }
  }
  if (a.kind == LF_VOXELS) {
    a.planes = planes_out;
    a.plane_dtype = dtype_out;
    PhaseScope ps(prof, LF_PHASE_FILTER, s);
    if ((e = launch_lowpass(a, s)) != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t build_planes(BuildArgs& a, const BuildLayout& L, hipStream_t s, Profiler* prof) {
  bool done = false;
  const hipError_t e = build_lists(a, L, s, prof, &done);
  if (e != hipSuccess || done) return e;
  return build_splat(a, L, s, prof);
}

hipError_t splat_batch_launch(const BuildArgs* args, const SplatJobs& jobs, int plane_dtype, hipStream_t s) {
  if (jobs.n < 1 || jobs.n > kMaxSplatJobs) return hipErrorInvalidValue;
  int64_t items = 0;
  for (int i = 0; i < jobs.n; ++i) items += jobs.max_items[i];
  const dim3 g((unsigned)xcd_grid(items, jobs.item_shift)), c((unsigned)kCombineGroups);
  hipLaunchKernelGGL(jobs_prefix, dim3(1), dim3(1), 0, s, args, jobs);
  switch (plane_dtype) {
    case LF_F16:
      hipLaunchKernelGGL((splat_gs_jobs<__half>), g, dim3(256), 0, s, args, jobs);
      hipLaunchKernelGGL((combine_jobs<__half>), c, dim3(256), 0, s, args, jobs);
      break;
    case LF_BF16:
      hipLaunchKernelGGL((splat_gs_jobs<__hip_bfloat16>), g, dim3(256), 0, s, args, jobs);
      hipLaunchKernelGGL((combine_jobs<__hip_bfloat16>), c, dim3(256), 0, s, args, jobs);
      break;
    case LF_U8:
      hipLaunchKernelGGL((splat_gs_jobs<uint8_t>), g, dim3(256), 0, s, args, jobs);
      hipLaunchKernelGGL((combine_jobs<uint8_t>), c, dim3(256), 0, s, args, jobs);
      break;
    default:
      hipLaunchKernelGGL((splat_gs_jobs<float>), g, dim3(256), 0, s, args, jobs);
      hipLaunchKernelGGL((combine_jobs<float>), c, dim3(256), 0, s, args, jobs);
      break;
  }
  return hipGetLastError();
}

hipError_t splat_work_launch(const BuildArgs& a, const BuildLayout& L, int64_t* counts, hipStream_t s) {
  hipError_t e = fill(reinterpret_cast<uint32_t*>(counts), 6, 0u, s);
  if (e != hipSuccess || a.n == 0) return e;
  // 64 partial triples in the radix sorts' scratch, which the build no longer needs
  unsigned long long* slots = reinterpret_cast<unsigned long long*>(a.radix_tmp);
  if ((e = fill(a.radix_tmp, 2 * 3 * 64, 0u, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(count_splat_work, dim3((unsigned)xcd_grid(L.max_items, a.item_shift)), dim3(256), 0, s, a, L.n_buckets,
                     slots);
  hipLaunchKernelGGL(sum_slots, dim3(1), dim3(64), 0, s, slots, reinterpret_cast<unsigned long long*>(counts));
  return hipGetLastError();
}

constexpr int kBwdItemShift = 12;

hipError_t build_backward(BuildArgs& a, const BuildLayout& L, hipStream_t s, Profiler* prof) {
  PhaseScope ps(prof, LF_PHASE_BUILD_BWD, s);
  hipError_t e;
  if (a.n == 0) return hipSuccess;
  if ((e = fill(reinterpret_cast<uint32_t*>(a.ggrad), a.n * kGradSlots, 0u, s)) != hipSuccess) return e;
  // The backward's work-groups add into per-Gaussian accumulators: with the chunk-major
  // items it ran fastest in 4096 blocks (1.21 ms at 200k Gaussians, against 1.77 ms in the
  // 256 blocks of the forward, where the work-groups in flight on an XCD share many
  // Gaussians, and 1.75 ms with one item per block).
  BuildArgs b = a;
  b.item_shift = kBwdItemShift;
  hipLaunchKernelGGL(splat_bwd_gs, dim3((unsigned)xcd_grid(L.max_items, b.item_shift)), dim3(256), 0, s, b, L.n_buckets);
  hipLaunchKernelGGL(preprocess_bwd_gs, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace lf
