// Internal declarations of the MPI build (workspace layout and kernel arguments).
#pragma once

#include "lf_internal.h"

namespace lf {

constexpr int kTileShift = 4;          // 16 x 16 texel tiles
constexpr int kTile = 1 << kTileShift;
constexpr int kTableChunk = 256;       // floats per table-upload launch

// Counters at the start of the workspace, read back by lf_build_stats.
struct BuildHeader {
  int64_t n_vis;
  int64_t entries;
  int64_t capacity;
  int32_t overflow;
  int32_t pad;
};

// One projected Gaussian (64 bytes, four 16-byte groups).
struct GRec {
  int32_t x0, y0, x1, y1;             // inclusive texel box of the support (x1 < x0: empty)
  float mx_hi, my_hi, mx_lo, my_lo;   // projected mean, double-float, texels
  float ca, cb, cc, l2o;              // log2(o G(d)) = l2o + ca dx^2 + cb dx dy + cc dy^2
  float rgb[3];
  float pad;
};

constexpr int kEntryPad = 8;          // readable entries past the end of the tile lists
constexpr int kSegment = 256;         // entries per splat work item (longer buckets are split)

struct BuildLayout {
  int64_t n, cap, n_buckets;
  int32_t K, ntx, nty, n_tiles, tile_bits, chunk_bits;
  size_t o_hdr, o_keys, o_vals, o_keys_alt, o_vals_alt, o_rec, o_ntiles_i, o_ntiles_r, o_chunk_r, o_offsets,
      o_scan64, o_chunk_start, o_edges, o_dtab, o_nseg, o_bucket, o_scan32, o_radix, o_ekeys, o_evals, o_ekeys_alt,
      o_evals_alt, o_pcnt, o_item_start, o_pslot, o_items, o_partial;
  int64_t max_items, max_partial;
  size_t total;
};

// Fixed part of the layout for n primitives, K planes and a wp x hp plane; cap entries.
BuildLayout build_layout(int64_t n, int32_t K, int32_t wp, int32_t hp, int64_t cap);

struct BuildArgs {
  int64_t n, capacity;
  int32_t K, ntx, binning, plane_dtype, chunk_bits;
  float d_focal32;
  Consts c;
  // field (Gaussians)
  const float *means, *log_scales, *quats, *opacity, *rgb;
  // outputs
  void* planes;
  float* depth;
  int32_t *chunk_of, *chunk_count;
  // workspace
  BuildHeader* hdr;
  uint32_t *keys, *vals, *keys_alt, *vals_alt;
  GRec* rec;
  uint32_t* ntiles_i;
  uint64_t* ntiles_r;
  uint32_t* chunk_r;
  uint64_t *offsets, *scan_tmp64;
  int64_t* chunk_start;
  float *edges, *dtab;
  uint32_t *nseg, *bucket, *scan_tmp32, *radix_tmp;
  uint32_t *ekeys, *evals, *ekeys_alt, *evals_alt;
  // splat work items: bucket segments and their partial (C, T) tiles
  uint32_t *pcnt, *item_start, *pslot;
  uint2* items;
  float4* partial;
  int64_t max_items;
};

struct TableChunk {
  int32_t offset, count;
  float v[kTableChunk];
};

hipError_t upload_table(float* dst, const float* host, int n, hipStream_t s);
hipError_t build_gaussians(BuildArgs& a, const BuildLayout& L, hipStream_t s, Profiler* prof);

}  // namespace lf
