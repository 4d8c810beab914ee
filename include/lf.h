/*
 * lf.h - C ABI of the MI355X sweeping-plane light-field renderer.
 *
 * The library turns an explicit radiance field (3D Gaussians or sparse voxels) into
 * N_chunk shared, view-independent premultiplied RGBA sweeping planes seen from one
 * reference camera, then swizzle-blends those planes front to back into many sheared
 * light-field views in one pass ("Real-time 3D Visualization of Radiance Fields on
 * Light Field Displays", Sec. 4 and Alg. 1).
 *
 * Conventions shared by every entry point
 *  - Pointer spaces: lf_camera, lf_view arrays, lf_geometry_info and the out-parameters
 *    of the *_workspace / *_stats / lf_geometry / lf_quilt_views calls are HOST memory.
 *    Every array inside lf_field and lf_mpi, every image and every workspace is DEVICE
 *    memory on the context's GPU.
 *  - Ownership: the caller allocates and frees all inputs, outputs, gradients and
 *    workspaces; the library frees nothing it did not allocate and owns only lf_ctx.
 *  - Asynchrony: device work is enqueued on the given stream (a hipStream_t passed as
 *    void*, NULL = the null stream) and returns without waiting, except the calls
 *    documented as synchronising.
 *  - Errors: every call returns an lf_status; arguments are validated on the host
 *    before anything is enqueued, so an invalid call has no device side effect.
 *    lf_last_error() returns a message for the last failing call on this thread.
 *  - Camera frame: the base camera looks along +z, x to the right, y down; R, t map
 *    world points p to base-camera coordinates R p + t.  Angles are full angles, radians.
 *  - Thread safety: one context per thread (or per stream).
 */
#ifndef LF_H
#define LF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LF_OK = 0,
  LF_ERR_INVALID_ARG = 1,   /* a null pointer, a size or an enum out of range         */
  LF_ERR_UNSUPPORTED = 2,   /* a valid request the library does not implement         */
  LF_ERR_CAPACITY = 3,      /* a workspace too small; the needed size is reported      */
  LF_ERR_OUT_OF_MEMORY = 4, /* a library-owned allocation failed                       */
  LF_ERR_HIP = 5            /* a HIP runtime call failed (also deferred async errors)  */
} lf_status;

/* LF_U8 (planes only): UNORM8, the default plane format of Sec. 5.1 (8-bit C and T):    
 * code = round-to-nearest-even(255 v) of the float32 value v clamped to [0, 1], read back
 * as code / 255.                                                                          */
typedef enum { LF_F32 = 0, LF_F16 = 1, LF_BF16 = 2, LF_U8 = 3 } lf_dtype;
typedef enum { LF_NEAREST = 0, LF_BILINEAR = 1 } lf_interp;
typedef enum { LF_BIN_QUANTILE = 0, LF_BIN_INV_DEPTH = 1 } lf_binning;
typedef enum { LF_GAUSSIANS = 0, LF_VOXELS = 1 } lf_field_kind;

#define LF_MAX_VIEWS 256          /* views per lf_composite call                         */
#define LF_MAX_CHUNKS 4096        /* sweeping planes per MPI                             */
#define LF_MAX_RES 8192           /* per-view and per-plane resolution limit             */

typedef struct lf_ctx lf_ctx;

/* The quilt parameters H of Alg. 1: base camera, display window and plane settings
 * (Sec. 4.2-4.3).  Host memory.                                                           */
typedef struct {
  float R[9];          /* world -> base camera rotation, row major                           */
  float t[3];          /* world -> base camera translation                                   */
  int32_t nx, ny;      /* per-view resolution N_x, N_y                                       */
  float fov_x, fov_y;  /* base camera field of view theta_x, theta_y (0 < theta < pi)        */
  float d_focal;       /* D_focal: base camera to focal-plane distance (> 0)                 */
  float phi_x, phi_y;  /* display viewing angles (0 <= phi < pi)                             */
  float d_shift;       /* D_shift: moves the reference camera back (Sec. 4.2), >= 0          */
  float plane_scale;   /* P_s: plane resolution = round(P_s * N)                             */
  float z_near;        /* primitives with reference depth <= z_near are culled (> 0)         */
  float dilation;      /* f' in reference texels^2: 0 = the adaptive value of Eq. 8; > 0 =
                        * this constant (the constant filter of the adaptive-filter ablation,
                        * Sec. 5)                                                             */
} lf_camera;

/* One quilt view: lateral offset of Eq. 4 in base-camera units.  The principal-point
 * shift of Eq. 5 is implied (principal rays meet the focal-plane centre).  Host memory. */
typedef struct { float dx, dy; } lf_view;

/* The radiance field P of Alg. 1.  Device memory, float32, C-contiguous.
 *  LF_GAUSSIANS: means[n][3], log_scales[n][3], quats[n][4] (w, x, y, z; normalised
 *                inside), opacity[n] (activated, in [0, 1]), rgb[n][3] (view-independent).
 *  LF_VOXELS:    ijk[n][3] int32 cell indices, density[n][8] corner densities per world
 *                unit (corner bit0 = +x, bit1 = +y, bit2 = +z), rgb[n][3]; the cell
 *                (i, j, k) spans origin + voxel_size * [i, i+1] x [j, j+1] x [k, k+1].    */
typedef struct {
  int32_t kind;
  int32_t reserved;
  int64_t n;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity;
  const float* rgb;
  const int32_t* ijk;
  const float* density;
  float origin[3];
  float voxel_size;
} lf_field;

/* Sweeping planes C, T of Sec. 4.2 as premultiplied RGBA (alpha = 1 - T_k).  Device.    */
typedef struct {
  int32_t dtype;          /* lf_dtype of rgba                                             */
  int32_t n_chunk;        /* K                                                            */
  int32_t height, width;  /* H_p = round(P_s N_y), W_p = round(P_s N_x)                   */
  void* rgba;             /* [n_chunk][height][width][4]                                  */
  float* depth;           /* [n_chunk] plane depths d_k (base-camera z)                   */
  int32_t* chunk_of;      /* [n] chunk per primitive, -1 = culled (may be NULL)           */
  int32_t* chunk_count;   /* [n_chunk] primitives per chunk (may be NULL)                 */
} lf_mpi;

/* Derived display geometry (Eqs. 1-2, 5, 8) - host values for inspection and tests.      */
typedef struct {
  double d_forward0;      /* Eq. 1                                                        */
  double d_forward;       /* Eq. 1 minus D_shift: reference camera position on +z         */
  double tan_half_theta_prime_x, tan_half_theta_prime_y;   /* Eq. 2                       */
  double f_dilation;      /* Eq. 8, reference texels^2                                    */
  double fpx, fpy, cpx, cpy;   /* reference intrinsics in plane texels                    */
  double fx, fy, cx, cy;       /* base-view intrinsics in pixels                          */
  int32_t plane_width, plane_height;
  /* float32 constants of the decision programs (bit patterns the kernels use)            */
  float d_forward32, guard_x32, guard_y32, ratio_x32, ratio_y32, fpx32, fpy32;
  float cpx32, cpy32, cx32, cy32, inv_focal32;
} lf_geometry_info;

typedef struct {
  int64_t n_visible;        /* primitives inside the reference frustum                    */
  int64_t entries_needed;   /* (tile, chunk) list entries the last build needed           */
  int64_t entry_capacity;   /* entries the workspace holds                                */
  int32_t overflow;         /* 1 if entries_needed > entry_capacity (planes are invalid)  */
  int32_t stalled;          /* 1 if a bounded device-wide wait of the sorts or scans gave
                             * up (planes are invalid; reported as LF_ERR_HIP)            */
} lf_build_info;

/* Gradients of a Gaussian field's parameters, device float32 arrays written whole by
 * lf_build_mpi_backward (culled Gaussians get zeros).                                    */
typedef struct {
  float* means;           /* [n][3]                                                       */
  float* log_scales;      /* [n][3]                                                       */
  float* quats;           /* [n][4], with respect to the un-normalised input quaternion   */
  float* opacity;         /* [n]                                                          */
  float* rgb;             /* [n][3]                                                       */
} lf_gaussian_grads;

/* Library version string.                                                               */
const char* lf_version(void);

/* Message of the last failing call on this thread ("" if none).                          */
const char* lf_last_error(void);

/* Create a context on HIP device `device`; fails with LF_ERR_HIP if it is absent.  The
 * context allocates (once, about 21 MB of device memory) the table of sampling
 * coefficients lf_composite and lf_composite_backward fill on their stream before they
 * composite, so those calls never allocate, free or synchronise and may be captured into
 * a graph.  Calls on one context share that table: calls that overlap on different
 * streams race (one context per stream).                                                 */
lf_status lf_create(lf_ctx** out, int device);
void lf_destroy(lf_ctx* ctx);

/* Derived geometry of a camera (Eqs. 1-2, 8; Sec. 4.2).  Host only, no GPU needed.       */
lf_status lf_geometry(const lf_camera* cam, lf_geometry_info* out);

/* View offsets of a vx-by-vy quilt, Eqs. 3-4 (row-major, s = 0 for a single row or
 * column).  Host only.  `out` holds vx * vy entries.                                     */
lf_status lf_quilt_views(const lf_camera* cam, int32_t vx, int32_t vy, lf_view* out);

/* Bytes of workspace lf_build_mpi needs for `field` with room for `entry_capacity`
 * (tile, chunk) list entries (entry_capacity <= 0 picks 16 per primitive, at least 65536). */
lf_status lf_build_mpi_workspace(const lf_field* field, const lf_camera* cam, int32_t n_chunk,
                                 int64_t entry_capacity, size_t* bytes);

/* Alg. 1 steps 1-5: cull and key, sort and chunk, rasterise every chunk into its plane.
 * Sec. 4.4 (Gaussians) / Sec. 4.5 (voxels, followed by the in-place plane low-pass).
 * binning: LF_BIN_QUANTILE (Sec. 4.4) or LF_BIN_INV_DEPTH with inv_depth_range = {z_lo,
 * z_hi} (host, z_lo > D_forward).  `mpi` describes caller-allocated outputs whose
 * n_chunk/width/height must match the camera; dtype may be F32, F16, BF16 or U8.
 * Enqueued on `stream` with no host synchronisation; if the workspace's entry capacity
 * is exceeded the planes are invalid and lf_build_stats reports it.                    */
lf_status lf_build_mpi(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, int32_t n_chunk,
                       int32_t binning, const float* inv_depth_range, lf_mpi* mpi,
                       void* workspace, size_t workspace_bytes, void* stream);

/* Counters of the last lf_build_mpi that used `workspace`.  SYNCHRONISES `stream`.
 * Returns LF_ERR_CAPACITY (with *out filled) if that build overflowed, LF_ERR_HIP (with
 * *out filled) if one of its bounded device-wide waits gave up.                          */
lf_status lf_build_stats(lf_ctx* ctx, const void* workspace, size_t workspace_bytes,
                         lf_build_info* out, void* stream);

/* The (tile, chunk) lists of the last lf_build_mpi on `workspace` (Sec. 4.4 and Alg. 1
 * "Rasterize": every chunk's primitives binned to the square tiles of the plane their
 * support box covers, each list in (depth key, index) order).  Diagnostic entry point for
 * tests.  field, cam, n_chunk: those of that build.  Host outputs: *tile (texels per tile
 * side), *tiles_x, *tiles_y.  Device outputs, each skipped when NULL (both NULL: only the
 * host outputs, no GPU work): bucket_start [tiles_x * tiles_y * n_chunk + 1] int64, the
 * list of chunk k in tile t = ty * tiles_x + tx being entries[bucket_start[t * n_chunk +
 * k] .. bucket_start[t * n_chunk + k + 1]) and bucket_start[last] the number of entries;
 * entries [entries_needed of lf_build_stats] int32 primitive indices.  A build that
 * overflowed its capacity has no lists (every start 0).  Enqueued on `stream`.            */
lf_status lf_build_tile_lists(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, int32_t n_chunk,
                              const void* workspace, size_t workspace_bytes, int32_t* tile, int32_t* tiles_x,
                              int32_t* tiles_y, int64_t* bucket_start, int32_t* entries, void* stream);

/* The splat's work in the last lf_build_mpi of a Gaussian field on `workspace` (Sec. 4.4,
 * Alg. 1 "Rasterize"; the blend of Eq. 7 within a chunk), counted with the splat's own
 * work items and float32 decisions.  Diagnostic entry point for measurement.  field, cam,
 * n_chunk: those of that build.  counts: device int64 [3], overwritten:
 *   counts[0] = support pairs: (Gaussian, plane texel) pairs with o G >= 1/255;
 *   counts[1] = (list entry, texel) evaluations the splat performs: every entry of a
 *               tile's list against the 64 texels of each 8x8 quadrant its 1/255 ellipse
 *               reaches;
 *   counts[2] = list entries x 256 texels (the whole tiles the lists name).
 * A build that overflowed its capacity counts zero.  Voxel fields: LF_ERR_UNSUPPORTED.
 * Enqueued on `stream`; needs the tile lists the build left in the workspace, and uses the
 * workspace's sort scratch (which nothing after the build reads, lf_build_mpi_backward
 * included) for partial counts.                                                         */
lf_status lf_build_splat_work(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, int32_t n_chunk,
                              const void* workspace, size_t workspace_bytes, int64_t* counts, void* stream);

/* The conventional per-view render that the light field approximates (the baseline of
 * Sec. 5.1, Table 1): every Gaussian of `field` in one depth-sorted chunk, splatted from
 * the camera of view `view` (Eq. 5: at (dx, dy, 0) in base-camera coordinates, looking
 * along +z, principal point shifted so its principal ray meets the focal-plane centre) at
 * the view resolution with the constant 0.3 px^2 dilation of 3DGS.  Culled: depth <=
 * z_near, or |x / z| > 1.3 tan(theta_x / 2) (view coordinates, about the view axis), or
 * likewise in y.  `out` is a one-plane MPI of the view size (n_chunk = 1, height = ny,
 * width = nx, any plane dtype): rgba = premultiplied (C, 1 - T), depth[0] = the median
 * depth; chunk_of / chunk_count may be NULL.  `workspace`: lf_render_view_workspace bytes
 * (reported by lf_build_stats like a build).  Gaussian fields only (voxels:
 * LF_ERR_UNSUPPORTED).  Enqueued on `stream`.                                            */
lf_status lf_render_view_workspace(const lf_field* field, const lf_camera* cam, size_t* bytes);
lf_status lf_render_view(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, const lf_view* view,
                         lf_mpi* out, void* workspace, size_t workspace_bytes, void* stream);

/* Swizzle blending (Sec. 4.3, Eqs. 6-7, Alg. 1 steps 6-11): for each view v, pixel (x, y)
 * and plane k front to back, sample plane k at the texel coordinate of Eq. 6 (nearest or
 * bilinear; outside the plane is transparent) and over-composite with float32
 * transmittance.  out: device [n_views][ny][nx][4] of (Q_r, Q_g, Q_b, T) in out_dtype
 * (F32 or F16).  views: host array of n_views (1..LF_MAX_VIEWS) offsets.                */
lf_status lf_composite(lf_ctx* ctx, const lf_mpi* mpi, const lf_camera* cam, const lf_view* views,
                       int32_t n_views, int32_t interp, int32_t out_dtype, void* out, void* stream);

/* lf_composite for callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and results, with
 * the coefficient table in a static device array of LF_COMPOSITE_SCRATCH_BYTES that each
 * GPU holds until the process ends (its address is resolved by lf_create).  The call
 * allocates nothing, host or device.  The table needs
 * 16 K V + 4 K (V + 24) + 8 K V bytes, each term rounded up to 256, plus 256, for K = mpi->n_chunk
 * planes and V = n_views views; a call beyond LF_COMPOSITE_SCRATCH_BYTES returns LF_ERR_CAPACITY
 * before anything is enqueued.  Every call on one GPU shares that one array (each call
 * rewrites it before compositing): calls that overlap on one GPU, on any streams or
 * contexts, race.  Arguments and outputs as lf_composite.                                */
#define LF_COMPOSITE_SCRATCH_BYTES (4u << 20)
lf_status lf_composite_noalloc(lf_ctx* ctx, const lf_mpi* mpi, const lf_camera* cam, const lf_view* views,
                               int32_t n_views, int32_t interp, int32_t out_dtype, void* out, void* stream);

/* Vector-Jacobian product of lf_composite (the over operator of Eq. 7 with the Eq. 6
 * sampling held fixed): given d_out = dL/d(Q_r, Q_g, Q_b, T) (device float32
 * [n_views][ny][nx][4]), writes d_planes = dL/d(C_r, C_g, C_b, A) (device float32
 * [n_chunk][height][width][4]; zero-filled by the callee, then accumulated).  The planes
 * of `mpi` are read in their own dtype (U8 planes: LF_ERR_UNSUPPORTED, the quantisation
 * has no gradient); per-pixel transmittance is recomputed, not stored.  Arguments as
 * lf_composite.                                                                           */
lf_status lf_composite_backward(lf_ctx* ctx, const lf_mpi* mpi, const lf_camera* cam, const lf_view* views,
                                int32_t n_views, int32_t interp, const float* d_out, float* d_planes,
                                void* stream);

/* Vector-Jacobian product of lf_build_mpi for a Gaussian field: given d_planes =
 * dL/d(C, A) of the planes (device float32 [n_chunk][height][width][4]), writes the
 * gradients of means, log-scales, quaternions, opacities and colours.  The partition, the
 * tile lists, the inclusion test o G >= 1/255 and the 0.99 clamp are held fixed (the
 * gradient of the smooth piece the parameters lie in; plane depths are constants).  It
 * reads the tile lists and per-Gaussian records that lf_build_mpi left in `workspace`, so
 * it must follow the lf_build_mpi call that produced `mpi` with the same field, camera,
 * n_chunk and workspace, with no other build on that workspace in between.  Voxel fields
 * return LF_ERR_UNSUPPORTED.                                                             */
lf_status lf_build_mpi_backward(lf_ctx* ctx, const lf_field* field, const lf_camera* cam, const lf_mpi* mpi,
                                const float* d_planes, const lf_gaussian_grads* grads, void* workspace,
                                size_t workspace_bytes, void* stream);

/* The float32 texel-coordinate coefficients lf_composite uses (Eq. 6 in affine form):
 * X = fl(fl(bx[k] * fl(x - c_x)) + Cx[k][v]) and Y likewise; the *_n offsets are the
 * nearest-sampling ones (floor(X) is the texel).  Device outputs: bx, by [n_chunk];
 * cx, cy, cxn, cyn [n_chunk][n_views].  Diagnostic entry point.                         */
lf_status lf_plane_coeffs(lf_ctx* ctx, const lf_mpi* mpi, const lf_camera* cam, const lf_view* views,
                          int32_t n_views, float* bx, float* by, float* cx, float* cy, float* cxn,
                          float* cyn, void* stream);

/* ---------------------------------------------------------------------------------------
 * Spherical-harmonic colour (the SH ablation of Sec. 5, Fig. 6).  A Gaussian may carry
 * real spherical-harmonic colour coefficients sh[n][(L+1)^2][3] (device float32, degree
 * L <= LF_MAX_SH_DEGREE, basis index j = l^2 + l + m, Condon-Shortley phase in the sign
 * convention of 3D Gaussian splatting); seen along the unit direction d its colour is
 * max(sum_j sh_j Y_j(d) + 1/2, 0).  SH planes keep per texel the coefficients blended
 * with the RGB planes' weights, q_j = sum_i alpha_i T_i sh_ij, and A = 1 - T, in
 * lf_sh_texel_floats(L) float32s: q_0 (r, g, b), A, q_1 (r, g, b), ..., q_{n-1} (r, g, b),
 * then zeros.  As everywhere in this header, the caller owns every buffer, and arguments
 * are validated on the host (LF_ERR_INVALID_ARG, with lf_last_error) before anything is
 * enqueued.
 * ------------------------------------------------------------------------------------- */
#define LF_MAX_SH_DEGREE 3

typedef struct {
  int32_t degree;         /* L, 0..LF_MAX_SH_DEGREE                                       */
  int32_t n_chunk;        /* K                                                            */
  int32_t height, width;  /* H_p, W_p as for lf_mpi                                       */
  float* planes;          /* [n_chunk][height][width][lf_sh_texel_floats(degree)]         */
  float* depth;           /* [n_chunk] plane depths d_k                                   */
} lf_sh_mpi;

/* Floats per SH-plane texel, 4 ceil((3 (L+1)^2 + 1) / 4) (4, 16, 28, 52); 0 for a degree
 * outside [0, LF_MAX_SH_DEGREE].  Host only.                                              */
int32_t lf_sh_texel_floats(int32_t degree);

/* Alg. 1 steps 1-5 with SH colour: the partition, tile lists and rasterisation of
 * lf_build_mpi for a Gaussian field, the planes blending `sh` (device [field->n][(L+1)^2]
 * [3]) instead of rgb (field->rgb may be NULL; it is not used).  The workspace is that of
 * lf_build_mpi (lf_build_mpi_workspace) and lf_build_stats reports on it.  Voxel fields:
 * LF_ERR_UNSUPPORTED.  Enqueued on `stream`.                                              */
lf_status lf_build_mpi_sh(lf_ctx* ctx, const lf_field* field, const float* sh, const lf_camera* cam,
                          int32_t n_chunk, int32_t binning, const float* inv_depth_range, lf_sh_mpi* mpi,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Swizzle blending of SH planes (Eqs. 6-7): plane k is sampled by view v at pixel (x, y)
 * as lf_composite samples it (nearest or bilinear, over all texel floats), and the sample
 * adds the premultiplied colour max(sum_j q_j Y_j(d) + A / 2, 0), d the world direction of
 * the pixel's ray in view v (Eq. 5 camera), the same for every plane.  out: device float32
 * [n_views][ny][nx][4] of (Q_r, Q_g, Q_b, T).  Other arguments as lf_composite.          */
lf_status lf_composite_sh(lf_ctx* ctx, const lf_sh_mpi* mpi, const lf_camera* cam, const lf_view* views,
                          int32_t n_views, int32_t interp, float* out, void* stream);

/* Colour of every Gaussian seen from view `view`: max(sum_j sh_j Y_j(d) + 1/2, 0), d the
 * unit direction from the view camera's centre (Eq. 5: (dx, dy, 0) in base-camera axes) to
 * the mean.  means [n][3], sh [n][(L+1)^2][3], rgb_out [n][3]: device float32.  With
 * lf_render_view on the field with rgb = rgb_out this is the per-view render in SH colour. */
lf_status lf_sh_colours(lf_ctx* ctx, const float* means, const float* sh, int32_t degree, int64_t n,
                        const lf_camera* cam, const lf_view* view, float* rgb_out, void* stream);

/* ---------------------------------------------------------------------------------------
 * Batches.  Several scenes (fields, cameras, plane counts, view lists) rendered by one
 * call.  By default each scene's build and composite go to a stream of their own, forked
 * from and joined back into the caller's stream, so small scenes run side by side on the
 * GPU.  With LF_BATCH_WORKLIST the batch runs phase by phase instead: each scene's cull,
 * depth sort, chunks and tile lists (Alg. 1 steps 1-4) on its own stream, then one splat
 * launch and one merge launch over the work items (tile, chunk segments) of every scene
 * with planes of one dtype, then one composite launch over the row tiles of every scene
 * with one kernel key (plane and view dtypes, sampling, view-group size); each phase's
 * kernel walks the (scene, item) list.  Voxel and empty fields build on their own streams,
 * and scenes that need the per-pixel composite or 256-pixel row tiles composite alone.
 * With LF_BATCH_GRAPH the first lf_batch_run captures the whole batch into a HIP graph and
 * every run (the first included) replays it with one launch.  With LF_BATCH_AUTOTUNE,
 * lf_batch_create times the composite of every scene with each view-group size (4, 8,
 * 12, 16 views per work-group) and row-tile width (64-pixel one-wave tiles, or 256-pixel
 * row-kernel tiles) and keeps the fastest (it builds each scene once and synchronises the
 * device); the choice is cached per process for the scene's camera, plane count and
 * dtype, views, sampling and output dtype, so a later batch of the same shapes is not
 * timed again.
 * ------------------------------------------------------------------------------------- */
typedef struct {
  lf_field field;           /* device field, as for lf_build_mpi                          */
  lf_camera cam;
  int32_t n_chunk;
  int32_t binning;          /* LF_BIN_QUANTILE or LF_BIN_INV_DEPTH                        */
  float inv_depth_range[2]; /* used with LF_BIN_INV_DEPTH                                 */
  const lf_view* views;     /* host array, copied by lf_batch_create                      */
  int32_t n_views;
  int32_t interp;           /* lf_interp                                                  */
  int32_t out_dtype;        /* F32 or F16                                                 */
  lf_mpi mpi;               /* caller-allocated planes (and optional chunk outputs)       */
  void* out;                /* caller-allocated views [n_views][ny][nx][4]                */
  void* workspace;          /* caller-allocated build workspace of this scene             */
  size_t workspace_bytes;
} lf_batch_item;

enum { LF_BATCH_GRAPH = 1, LF_BATCH_AUTOTUNE = 2, LF_BATCH_WORKLIST = 4 };

typedef struct lf_batch lf_batch;

/* Validates and records n_items scenes (1..LF_MAX_BATCH).  Every device buffer an item
 * names must stay valid, and keep its address, while the batch is used.                  */
#define LF_MAX_BATCH 64
lf_status lf_batch_create(lf_ctx* ctx, const lf_batch_item* items, int32_t n_items, int32_t flags,
                          lf_batch** out);

/* Renders every scene (build then composite) on `stream`.  Asynchronous; lf_batch_stats
 * reports the builds' capacity overflows and timed-out waits after it.                   */
lf_status lf_batch_run(lf_batch* batch, void* stream);

/* Build counters of every scene of the batch's last run, as lf_build_stats gives them for
 * one build: out, if not NULL, a host array of the batch's n_items entries; *n_failed, if
 * not NULL, the number of scenes whose build overflowed its entry capacity or gave up a
 * bounded device-wide wait (their planes and views are invalid).  SYNCHRONISES `stream`
 * (the stream of the run).  Returns LF_ERR_HIP if a scene's wait gave up, else
 * LF_ERR_CAPACITY if a scene overflowed (the message names the first such scene), else
 * LF_OK; out and n_failed are filled in every case.                                      */
lf_status lf_batch_stats(lf_batch* batch, lf_build_info* out, int32_t* n_failed, void* stream);

/* The view-group size the composite of scene `item` uses (autotuned, or 0 for default). */
lf_status lf_batch_group(const lf_batch* batch, int32_t item, int32_t* group);

/* The row-tile width the composite of scene `item` uses (64 or 256 autotuned, or 0 for
 * default: 64-pixel one-wave tiles where the windows fit).                               */
lf_status lf_batch_tile(const lf_batch* batch, int32_t item, int32_t* tile);

void lf_batch_destroy(lf_batch* batch);

/* Per-phase device timing, a tracing aid.  While enabled, each entry point brackets its
 * kernel phases with HIP events recorded on the launch stream; lf_profile_read sums the
 * elapsed times.  Phases: PREPROCESS (cull, key, projection), SORT (depth sort), BIN
 * (chunking, tile lists), SPLAT (the plane rasterisation kernel alone), MERGE (over-
 * composition of split tile lists), FILTER (voxel plane low-pass), COEFF (per-plane,
 * per-view sampling coefficients), COMPOSITE (the swizzle-blend kernel alone), and the
 * two backward passes.                                                                  */
typedef enum {
  LF_PHASE_PREPROCESS = 0, LF_PHASE_SORT = 1, LF_PHASE_BIN = 2, LF_PHASE_SPLAT = 3,
  LF_PHASE_MERGE = 4, LF_PHASE_FILTER = 5, LF_PHASE_COEFF = 6, LF_PHASE_COMPOSITE = 7,
  LF_PHASE_COMPOSITE_BWD = 8, LF_PHASE_BUILD_BWD = 9, LF_NUM_PHASES = 10
} lf_phase;

lf_status lf_profile_enable(lf_ctx* ctx, int32_t enable);

/* Milliseconds summed per phase and the number of bracketed launches since the last reset
 * (host arrays of LF_NUM_PHASES).  SYNCHRONISES the device.                             */
lf_status lf_profile_read(lf_ctx* ctx, double* ms, int64_t* count, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* LF_H */
