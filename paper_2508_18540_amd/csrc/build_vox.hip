// Sparse-voxel kernels of the MPI build (V2LF, Sec. 4.5) for gfx950.  The voxels go through
// the same cull / sort / chunk / tile-list pipeline as Gaussians (build_gs.hip); only the
// per-primitive preprocess, the splat and the plane low-pass differ.
//
//  preprocess  per voxel: float32 centre fl(o + fl(h fl(i + 1/2))), its depth key and cull
//              (the Gaussian program), the reference camera centre in the cube's local
//              units, and the texel box of the eight projected corners widened by one texel
//  splat       one work-group per (tile, chunk) item, one wave per 8x8 texel quadrant
//              walking the bucket with scalar loads (as for Gaussians).  Per texel ray
//              u(t) = a + t b in cube units: slab interval [t0, t1] (t >= 0); the trilinear
//              density along the ray is a cubic in t, so a 2-point Gauss-Legendre rule gives
//              its integral exactly: tau = |r| (t1 - t0)/2 (rho(u+) + rho(u-)); alpha =
//              1 - exp(-tau); front to back C += T alpha rgb, T *= 1 - alpha
//  low-pass    separable [1, 2, 1] / 4 with zero padding, in place: the original rows and
//              columns bordering every 16 x 64 region are saved first, then each region is
//              filtered from its own texels and the saved border
#include "build_device.h"

namespace lf {
namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kInvSqrt3 = 0.57735026918962576f;

__global__ __launch_bounds__(256) void preprocess_vox(BuildArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Consts& c = a.c;
  const int ix = a.ijk[3 * i], iy = a.ijk[3 * i + 1], iz = a.ijk[3 * i + 2];
  const float fx = (float)ix, fy = (float)iy, fz = (float)iz;
  const float h = a.vsize;
  const float mx = a.origin[0] + h * (fx + 0.5f);
  const float my = a.origin[1] + h * (fy + 0.5f);
  const float mz = a.origin[2] + h * (fz + 0.5f);
  const KeyCull kc = key_and_cull(c, mx, my, mz);
  a.keys[i] = kc.vis ? orderable(kc.key) : 0xffffffffu;
  a.vals[i] = (uint32_t)i;
  a.ntiles_i[i] = 0;
  if (a.chunk_of) a.chunk_of[i] = -1;
  if (!kc.vis) return;

  VRec r;
  // reference camera centre relative to the cube's low corner, in cell units (double-float in)
  r.ax = (a.cam_cell[0] - fx) + a.cam_cell_lo[0];
  r.ay = (a.cam_cell[1] - fy) + a.cam_cell_lo[1];
  r.az = (a.cam_cell[2] - fz) + a.cam_cell_lo[2];
  r.pad0 = 0.0f;
  for (int q = 0; q < 8; ++q) r.dens[q] = a.density[8 * i + q];
  r.rgb[0] = a.rgb[3 * i];
  r.rgb[1] = a.rgb[3 * i + 1];
  r.rgb[2] = a.rgb[3 * i + 2];
  r.pad1 = 0.0f;

  // texel box: the projected corners' bounding box, widened by one texel for rounding
  const float lx = a.origin[0] + h * fx, ly = a.origin[1] + h * fy, lz = a.origin[2] + h * fz;
  float X0 = INFINITY, X1 = -INFINITY, Y0 = INFINITY, Y1 = -INFINITY;
  bool behind = false;
  for (int q = 0; q < 8; ++q) {
    const float px = lx + ((q & 1) ? h : 0.0f), py = ly + ((q & 2) ? h : 0.0f), pz = lz + ((q & 4) ? h : 0.0f);
    const float cx = ((c.R[0] * px + c.R[1] * py) + c.R[2] * pz) + c.t[0];
    const float cy = ((c.R[3] * px + c.R[4] * py) + c.R[5] * pz) + c.t[1];
    const float zr = (((c.R[6] * px + c.R[7] * py) + c.R[8] * pz) + c.t[2]) - c.d_fwd;
    if (!(zr > 0.0f)) {
      behind = true;
      continue;
    }
    const float X = c.fpx * cx / zr + c.cpx, Y = c.fpy * cy / zr + c.cpy;
    X0 = fminf(X0, X);
    X1 = fmaxf(X1, X);
    Y0 = fminf(Y0, Y);
    Y1 = fmaxf(Y1, Y);
  }
  r.x0 = r.y0 = 0;
  r.x1 = r.y1 = -1;
  float fx0, fx1, fy0, fy1;
  if (behind) {
    fx0 = 0.0f;
    fy0 = 0.0f;
    fx1 = (float)(c.wp - 1);
    fy1 = (float)(c.hp - 1);
  } else {
    fx0 = fmaxf(floorf(X0) - 1.0f, 0.0f);
    fx1 = fminf(ceilf(X1) + 1.0f, (float)(c.wp - 1));
    fy0 = fmaxf(floorf(Y0) - 1.0f, 0.0f);
    fy1 = fminf(ceilf(Y1) + 1.0f, (float)(c.hp - 1));
  }
  uint32_t nt = 0;
  if (fx0 <= fx1 && fy0 <= fy1) {
    r.x0 = (int)fx0;
    r.x1 = (int)fx1;
    r.y0 = (int)fy0;
    r.y1 = (int)fy1;
    nt = box_tiles(r.x0, r.y0, r.x1, r.y1);
  }
  reinterpret_cast<VRec*>(a.rec)[i] = r;
  a.ntiles_i[i] = nt;
}

// trilinear interpolation of the corner densities at local coordinates (x, y, z)
__device__ __forceinline__ float trilerp(const float* d, float x, float y, float z) {
  const float c00 = fmaf(x, d[1] - d[0], d[0]), c10 = fmaf(x, d[3] - d[2], d[2]);
  const float c01 = fmaf(x, d[5] - d[4], d[4]), c11 = fmaf(x, d[7] - d[6], d[6]);
  const float c0 = fmaf(y, c10 - c00, c00), c1 = fmaf(y, c11 - c01, c01);
  return fmaf(z, c1 - c0, c0);
}

__device__ __forceinline__ float away_from_zero(float b) { return copysignf(fmaxf(fabsf(b), 1e-20f), b); }

template <typename PT>
__global__ __launch_bounds__(256) void splat_vox(BuildArgs a, int64_t n_buckets) {
  const uint32_t item = blockIdx.x;
  if (item >= a.item_start[n_buckets]) return;
  const uint2 it = a.items[item];
  const int64_t bidx = it.x;
  const int tile = (int)(bidx / a.K), k = (int)(bidx % a.K);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ox = (tile % a.ntx) << kTileShift, oy = (tile / a.ntx) << kTileShift;
  const int px = ox + ((wave & 1) << 3) + (lane & 7), py = oy + ((wave >> 1) << 3) + (lane >> 3);
  const Consts& c = a.c;
  // the texel's reference ray r = ((x - c'x)/f'x, (y - c'y)/f'y, 1) in world cell units
  const float rx = ((float)px - c.cpx) / c.fpx, ry = ((float)py - c.cpy) / c.fpy;
  const float rn = sqrtf(fmaf(rx, rx, fmaf(ry, ry, 1.0f)));
  const float bx = away_from_zero(((c.R[0] * rx + c.R[3] * ry) + c.R[6]) * a.inv_vsize);
  const float by = away_from_zero(((c.R[1] * rx + c.R[4] * ry) + c.R[7]) * a.inv_vsize);
  const float bz = away_from_zero(((c.R[2] * rx + c.R[5] * ry) + c.R[8]) * a.inv_vsize);
  const float ibx = 1.0f / bx, iby = 1.0f / by, ibz = 1.0f / bz;
  const uint32_t* __restrict__ ev = a.evals;
  const VRec* __restrict__ rec = reinterpret_cast<const VRec*>(a.rec);
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
  const bool ok = a.hdr->overflow == 0;
  const uint32_t bb0 = a.bucket[bidx], bb1 = a.bucket[bidx + 1];
  const uint32_t nseg = seg_count(bb1 - bb0);
  if (ok) {
    const uint32_t b0 = bb0 + it.y * kSegment;
    const uint32_t b1 = min(bb1, b0 + kSegment);
    const uint32_t qbit = 1u << (28 + wave);
    for (uint32_t e = b0; e < b1; ++e) {
      const uint32_t ent = ev[e];
      if (!(ent & qbit)) continue;                            // scalar: the box misses this quadrant
      const VRec& v = rec[min(ent & 0x0fffffffu, (uint32_t)a.n - 1u)];
      // slab interval of u(t) = a + t b in [0, 1]^3, t >= 0
      const float tax = -v.ax * ibx, tay = -v.ay * iby, taz = -v.az * ibz;
      const float tbx = tax + ibx, tby = tay + iby, tbz = taz + ibz;
      const float t0 = fmaxf(fmaxf(fminf(tax, tbx), fminf(tay, tby)), fmaxf(fminf(taz, tbz), 0.0f));
      const float t1 = fminf(fminf(fmaxf(tax, tbx), fmaxf(tay, tby)), fmaxf(taz, tbz));
      const float mid = 0.5f * (t0 + t1), half = 0.5f * (t1 - t0);
      const float ux = fmaf(mid, bx, v.ax), uy = fmaf(mid, by, v.ay), uz = fmaf(mid, bz, v.az);
      const float g = half * kInvSqrt3;
      const float dx = g * bx, dy = g * by, dz = g * bz;
      const float rho = trilerp(v.dens, ux + dx, uy + dy, uz + dz) + trilerp(v.dens, ux - dx, uy - dy, uz - dz);
      const float tau = rn * half * rho;
      // rays that miss get alpha 0 (a select: the missed lanes' values are never used)
      const float alpha = t1 > t0 ? 1.0f - __builtin_amdgcn_exp2f(-kLog2e * tau) : 0.0f;
      const float w = alpha * T;
      C0 = fmaf(w, v.rgb[0], C0);
      C1 = fmaf(w, v.rgb[1], C1);
      C2 = fmaf(w, v.rgb[2], C2);
      T = T - w;
    }
  }
  if (nseg > 1) {
    const size_t slot = (size_t)a.pslot[bidx] + it.y;
    a.partial[slot * (kTile * kTile) + ((py - oy) << kTileShift) + (px - ox)] = make_float4(C0, C1, C2, T);
  } else if (px < c.wp && py < c.hp) {
    store_rgba(static_cast<PT*>(a.planes), ((size_t)k * c.hp + py) * c.wp + px, C0, C1, C2, 1.0f - T);
  }
}

// ---------------------------------------------------------------------------------------
// Low-pass: the separable [1, 2, 1] / 4 filter of every premultiplied channel, zero outside
// the plane, from the float32 stage into the planes (stored once, in their dtype).  One
// work-group per kFiltRows x kFiltCols region of one plane stages the region and its
// one-texel border in LDS.
// ---------------------------------------------------------------------------------------
template <typename PT>
__global__ __launch_bounds__(256) void lowpass(BuildArgs a) {
  constexpr int LR = kFiltRows + 2, LC = kFiltCols + 2;
  __shared__ float4 tile[LR][LC];
  const int seg = blockIdx.x, band = blockIdx.y, k = blockIdx.z;
  const int W = a.c.wp, H = a.c.hp;
  const int x0 = seg * kFiltCols, y0 = band * kFiltRows;
  const float4* __restrict__ src = a.stage + (size_t)k * H * W;
  for (int i = threadIdx.x; i < LR * LC; i += blockDim.x) {
    const int ly = i / LC, lx = i % LC;
    const int y = y0 - 1 + ly, x = x0 - 1 + lx;
    tile[ly][lx] = (x >= 0 && x < W && y >= 0 && y < H) ? src[(size_t)y * W + x] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  PT* planes = static_cast<PT*>(a.planes);
  for (int i = threadIdx.x; i < kFiltRows * kFiltCols; i += blockDim.x) {
    const int ly = i / kFiltCols + 1, lx = i % kFiltCols + 1;
    const int y = y0 + ly - 1, x = x0 + lx - 1;
    if (y >= H || x >= W) continue;
    float4 row[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float4 l = tile[ly - 1 + d][lx - 1], m = tile[ly - 1 + d][lx], r = tile[ly - 1 + d][lx + 1];
      row[d] = make_float4(0.25f * l.x + 0.5f * m.x + 0.25f * r.x, 0.25f * l.y + 0.5f * m.y + 0.25f * r.y,
                           0.25f * l.z + 0.5f * m.z + 0.25f * r.z, 0.25f * l.w + 0.5f * m.w + 0.25f * r.w);
    }
    const float4 o = make_float4(0.25f * row[0].x + 0.5f * row[1].x + 0.25f * row[2].x,
                                 0.25f * row[0].y + 0.5f * row[1].y + 0.25f * row[2].y,
                                 0.25f * row[0].z + 0.5f * row[1].z + 0.25f * row[2].z,
                                 0.25f * row[0].w + 0.5f * row[1].w + 0.25f * row[2].w);
    store_rgba(planes, ((size_t)k * H + y) * W + x, o.x, o.y, o.z, o.w);
  }
}

template <typename PT>
hipError_t lowpass_typed(const BuildArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((lowpass<PT>), dim3(a.filt_segs, a.filt_bands, a.K), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_preprocess_vox(const BuildArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(preprocess_vox, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_splat_vox(const BuildArgs& a, const BuildLayout& L, hipStream_t s) {
  const dim3 grid((unsigned)L.max_items);
  switch (a.plane_dtype) {
    case LF_F16: hipLaunchKernelGGL((splat_vox<__half>), grid, dim3(256), 0, s, a, L.n_buckets); break;
    case LF_BF16: hipLaunchKernelGGL((splat_vox<__hip_bfloat16>), grid, dim3(256), 0, s, a, L.n_buckets); break;
    case LF_U8: hipLaunchKernelGGL((splat_vox<uint8_t>), grid, dim3(256), 0, s, a, L.n_buckets); break;
    default: hipLaunchKernelGGL((splat_vox<float>), grid, dim3(256), 0, s, a, L.n_buckets); break;
  }
  return hipGetLastError();
}

hipError_t launch_lowpass(const BuildArgs& a, hipStream_t s) {
  if (a.K == 0 || a.c.wp == 0 || a.c.hp == 0) return hipSuccess;
  switch (a.plane_dtype) {
    case LF_F16: return lowpass_typed<__half>(a, s);
    case LF_BF16: return lowpass_typed<__hip_bfloat16>(a, s);
    case LF_U8: return lowpass_typed<uint8_t>(a, s);
    default: return lowpass_typed<float>(a, s);
  }
}

}  // namespace lf
