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
  uint32_t stalled;                   // a device-wide wait of the sorts or scans gave up
};

// One projected Gaussian (64 bytes, four 16-byte groups).
struct GRec {
  int32_t x0, y0, x1, y1;             // inclusive texel box of the support (x1 < x0: empty)
  float mx_hi, my_hi, mx_lo, my_lo;   // projected mean, double-float, texels
  float ca, cb, cc, l2o;              // log2(o G(d)) = l2o + ca dx^2 + cb dx dy + cc dy^2
  float rgb[3];
  float pad;
};

// One sparse voxel (80 bytes).  The box comes first, as in GRec, so the shared tile-list
// code reads both record kinds through the same first 16 bytes.
struct VRec {
  int32_t x0, y0, x1, y1;             // inclusive texel box of every ray that can meet the cube
  float ax, ay, az, pad0;             // reference-camera centre in the cube's local units (world)
  float dens[8];                      // corner densities (bit 0 = +x, bit 1 = +y, bit 2 = +z)
  float rgb[3];
  float pad1;
};

// Low-pass filter (voxel planes): regions of kFiltRows x kFiltCols texels, read from the
// float32 stage the voxel splat writes and stored into the planes in their dtype.
constexpr int kFiltRows = 16;
constexpr int kFiltCols = 64;

constexpr int kEntryPad = 8;          // readable entries past the end of the tile lists
constexpr int kSegment = 256;         // entries per splat work item (longer buckets are split)

struct BuildLayout {
  int64_t n, cap, n_buckets;
  int32_t K, ntx, nty, n_tiles, tile_bits, chunk_bits, kind, rec_bytes;
  int32_t filt_bands, filt_segs;      // voxel low-pass regions (0 for Gaussians)
  size_t o_hdr, o_keys, o_vals, o_keys_alt, o_vals_alt, o_rec, o_ntiles_i, o_ntiles_r, o_chunk_r, o_offsets,
      o_sync, o_chunk_start, o_edges, o_dtab, o_nseg, o_bucket, o_radix, o_ekeys, o_evals, o_ekeys_alt, o_heads,
      o_evals_alt, o_pcnt, o_item_start, o_pslot, o_split, o_items, o_partial, o_stage, o_ggrad;
  int64_t max_items, max_partial;
  // zero-initialised synchronisation words after the header (digit totals of both sorts,
  // scan states); the build clears [o_hdr, o_hdr + 4 clear_words) first
  int64_t clear_words;
  size_t total;
};

// log2 of the number of blocks the splat's work items are dealt to the XCDs in
// (LF_SPLAT_ITEM_SHIFT overrides it, 0..24)
int splat_item_shift();

// Fixed part of the layout for n primitives of `kind`, K planes and a wp x hp plane; cap
// entries.
BuildLayout build_layout(int32_t kind, int64_t n, int32_t K, int32_t wp, int32_t hp, int64_t cap);

struct BuildArgs {
  int64_t n, capacity;
  int32_t K, ntx, n_tiles, binning, plane_dtype, chunk_bits, kind, rec_bytes;
  float d_focal32;
  Consts c;
  // field (Gaussians)
  const float *means, *log_scales, *quats, *opacity, *rgb;
  // spherical-harmonic colour [n][sh_coef][3] (SH planes of float32 texels) or none (sh_coef 0)
  const float* sh;
  int32_t sh_coef;
  // field (voxels): cells, corner densities, grid origin and cell size; the reference camera
  // centre in world cell units, (R^T ((0, 0, D_fwd) - t) - origin) / h, as double-float
  const int32_t* ijk;
  const float* density;
  float origin[3], vsize, inv_vsize;
  float cam_cell[3], cam_cell_lo[3];
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
  uint64_t* offsets;
  int64_t* chunk_start;
  float *edges, *dtab;
  uint32_t *nseg, *bucket, *radix_tmp;
  // cleared at the start of every build: digit totals of the two sorts, scan states
  uint32_t *ghist_key, *ghist_tile;
  uint64_t *scan_state_offsets, *scan_state_items;
  int64_t clear_words;
  uint32_t *ekeys, *evals, *ekeys_alt, *evals_alt;
  // heads[b]: rank whose tile entries hold entry 256 b (written by the offsets scan)
  uint32_t* heads;
  int64_t n_heads;
  // splat work items: bucket segments and their partial (C, T) tiles
  uint32_t *pcnt, *item_start, *pslot;
  uint32_t* split;                    // per partial slot: its bucket if first of a split bucket, else ~0
  uint2* items;
  float4* partial;
  int64_t max_items;
  int32_t item_shift;                 // the splat's items go to the XCDs in 2^item_shift blocks
  // voxel planes: float32 stage [K][hp][wp] of the splat, filtered into the planes
  float4* stage;
  int32_t filt_bands, filt_segs;
  // backward: plane cotangents, per-Gaussian accumulators [n][kGradSlots], outputs
  const float* d_planes;
  float* ggrad;
  lf_gaussian_grads grads;
};

// Per-Gaussian accumulators of the splat backward: d/d(ca, cb, cc) of the log2-domain
// conic, d/d(projected mean x, y), d/d(log2 o), d/d(rgb).
constexpr int kGradSlots = 9;

struct TableChunk {
  int32_t offset, count;
  float v[kTableChunk];
};

hipError_t upload_table(float* dst, const float* host, int n, hipStream_t s);
// The whole build of one field (either kind) on stream s.
hipError_t build_planes(BuildArgs& a, const BuildLayout& L, hipStream_t s, Profiler* prof);
// Validates a build, derives its layout and kernel arguments and uploads its inverse-depth
// tables on st: what lf_build_mpi does before it launches (mpi: RGB planes, or with sh_coef
// > 0 float32 SH planes).
lf_status build_prepare(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, int32_t n_chunk, int32_t binning,
                        const float* inv_depth_range, const lf_mpi* mpi, const float* sh, int32_t sh_coef,
                        void* workspace, size_t workspace_bytes, hipStream_t st, BuildArgs* a, BuildLayout* L);
// build_planes in two parts: the cull, sort, chunks, tile lists and work items (*done: the
// planes are complete already, an empty field), then the splat and merge.  build_lists
// leaves a.evals on the entries' final array.
hipError_t build_lists(BuildArgs& a, const BuildLayout& L, hipStream_t s, Profiler* prof, bool* done);
hipError_t build_splat(BuildArgs& a, const BuildLayout& L, hipStream_t s, Profiler* prof);
// The splat and merge of several Gaussian builds (RGB planes of one dtype) in one launch
// each, over the work items of all of them: args [0 .. n) in device memory, each build's
// lists complete.
constexpr int kMaxSplatJobs = LF_MAX_BATCH;
struct SplatJobs {
  int32_t n;
  int32_t item_shift;                 // as BuildArgs::item_shift, over the joined item list
  uint32_t* prefix;                   // device scratch of 2 n + 2 words (the launch fills it)
  int64_t n_buckets[kMaxSplatJobs];
  int64_t max_items[kMaxSplatJobs];
};
hipError_t splat_batch_launch(const BuildArgs* args, const SplatJobs& jobs, int plane_dtype, hipStream_t s);
// Copies the (tile, chunk) bucket starts and the entries' primitive indices of the last build
// (a.evals must name the array the tile sort ended in); either output may be null.
hipError_t tile_lists_launch(const BuildArgs& a, const BuildLayout& L, int64_t* bucket_start, int32_t* entries,
                             hipStream_t s);
// Digit width the tile sort of the entries uses (its pass count decides where they end up).
int tile_digit_bits();

// Voxel kernels (build_vox.hip): per-voxel preprocess, tile-list splat of one plane per
// (tile, chunk) item, and the in-place plane low-pass.
hipError_t launch_preprocess_vox(const BuildArgs& a, hipStream_t s);
hipError_t launch_splat_vox(const BuildArgs& a, const BuildLayout& L, hipStream_t s);
hipError_t launch_lowpass(const BuildArgs& a, hipStream_t s);

// Backward of the Gaussian build (build_gs.hip): splat VJP into the per-Gaussian
// accumulators, then the projection's chain rule into the parameter gradients.
hipError_t build_backward(BuildArgs& a, const BuildLayout& L, hipStream_t s, Profiler* prof);
// counts[3] (int64) of the splat's work over the tile lists of the last build
hipError_t splat_work_launch(const BuildArgs& a, const BuildLayout& L, int64_t* counts, hipStream_t s);

}  // namespace lf
