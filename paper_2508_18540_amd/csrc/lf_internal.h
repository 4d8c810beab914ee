// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "lf.h"

namespace lf {

// HIP-event timing of kernel phases (enabled per context).
struct Profiler {
  struct Rec {
    int phase;
    hipEvent_t a, b;
  };
  bool on = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double ms[LF_NUM_PHASES] = {};
  int64_t count[LF_NUM_PHASES] = {};
  hipEvent_t take();
  size_t begin(int phase, hipStream_t s);   // returns the record's index for end()
  void end(size_t rec, hipStream_t s);
  hipError_t collect();
  void release();
};

// RAII bracket of one phase; a no-op when profiling is off or p is null.
struct PhaseScope {
  Profiler* p;
  hipStream_t s;
  size_t rec = 0;
  PhaseScope(Profiler* prof, int phase, hipStream_t st) : p(prof && prof->on ? prof : nullptr), s(st) {
    if (p) rec = p->begin(phase, s);
  }
  ~PhaseScope() {
    if (p) p->end(rec, s);
  }
};

}  // namespace lf

// Library context: the device it was created on and its profiler.
struct lf_ctx {
  int device;
  lf::Profiler prof;
  void* table = nullptr;         // device table of the composite's sampling coefficients,
  size_t table_bytes = 0;        // allocated by lf_create for the largest call
};

namespace lf {

// Float32 constants of the decision programs and of the projection.  The host derives
// every value in float64 (Eqs. 1-2, 8) and rounds it once; *_lo members hold the
// rounding residual (value - hi) so kernels can form double-float products.
struct Consts {
  float d_fwd, d_fwd_lo;     // reference camera position on the base camera's +z axis
  float z_near;
  float guard_x, guard_y;    // fl32(1.3 tan(theta'/2))
  float ratio_x, ratio_y;    // fl32(f'/f): plane texels per view pixel at unit magnification
  float fpx, fpx_lo, fpy, fpy_lo;   // reference focal lengths in texels
  float cpx, cpy;            // reference principal point (W_p - 1)/2, (H_p - 1)/2
  float cx, cy;              // view principal point (N - 1)/2
  float inv_focal;           // fl32(1 / D_focal)
  float f_dil;               // Eq. 8 dilation, texels^2
  float R[9], t[3];          // world -> base camera
  int32_t nx, ny, wp, hp;
};

struct Geom {
  double tx, ty, taux, tauy, d_forward0, d_forward, tpx, tpy;
  double fx, fy, cx, cy, fpx, fpy, cpx, cpy, f_dil;
  int32_t nx, ny, wp, hp;
  Consts c;
};

// Validates `cam` and derives its geometry.  Sets the thread's error message on failure.
lf_status derive_geometry(const lf_camera* cam, Geom* g);

// Thread-local error message helpers.
lf_status fail(lf_status s, const char* fmt, ...);
lf_status hip_fail(hipError_t e, const char* what);

// Eq. 6 in affine form for the plane at base depth d (see the composite kernels):
// X = bx (x - c_x) + c'_x + gx dx, Y = by (y - c_y) + c'_y + gy dy, in float32.
struct PlaneCo {
  float bx, by, gx, gy;
};

__device__ __forceinline__ PlaneCo plane_co(float d, const Consts& c) {
  const float z = d - c.d_fwd;
  const float q = d / z;
  const float w = (1.0f - d * c.inv_focal) / z;
  return {c.ratio_x * q, c.ratio_y * q, c.fpx * w, c.fpy * w};
}

struct CompositeArgs {
  const void* planes;
  const float* depth;
  void* out;
  int32_t K, hp, wp, nx, ny, n_views;
  int32_t plane_dtype, out_dtype, interp;
  int32_t group;            // views per row work-group (4, 8, 12, 16); 0 picks by view count
  int32_t tile;             // pixels per row tile: 64 (one wave, where the window fits; also 0)
                            // or 256 (every segment to the 256-thread row kernel)
  uint32_t* spill;          // set by the launch, in the coefficient table: the table kernel
                            // clears it, a one-wave work-group that leaves its segment to the
                            // row kernel sets it, and the row kernel returns at once while it
                            // is clear
  Consts c;
  float dx[LF_MAX_VIEWS];
  float dy[LF_MAX_VIEWS];
  // View groups of the row kernels, filled by the launch: views that share dy, listed class
  // by class in perm (position -> view index); vgroup[g] = first position | count << 8.
  int32_t n_groups;
  uint16_t vgroup[LF_MAX_VIEWS];
  uint8_t perm[LF_MAX_VIEWS];
};
static_assert(LF_MAX_VIEWS <= 256, "view positions and group starts are 8-bit");

// One scene's composite inside a batch launch: its arguments (view groups filled), its
// coefficient table (filled on the scene's stream beforehand), its 64-pixel segments per
// row and its tile count n_groups * nseg * ny.
struct CompositeJob {
  CompositeArgs a;
  const float4* pt;
  const float* ct;
  const float2* pm;
  int32_t nseg, tiles;
};
constexpr int kMaxJobs = LF_MAX_BATCH;
// Kernel key of a batch launch: scenes that share it composite in one launch.
struct CompositeKey {
  int32_t plane_dtype, out_dtype, interp, group;
  bool operator==(const CompositeKey& o) const {
    return plane_dtype == o.plane_dtype && out_dtype == o.out_dtype && interp == o.interp && group == o.group;
  }
};
// Prepares scene job j of a batch: picks the view-group size (a.group, else by view count),
// fills the view groups and the table's pointers; returns false if the scene needs the
// per-pixel kernel (then composite_launch serves it alone).
bool composite_job(CompositeArgs& a, void* table, CompositeJob* j, CompositeKey* key);
// Enqueues the coefficient table of a prepared job on s.
hipError_t composite_job_table(const CompositeJob& j, hipStream_t s);
// One launch of the one-wave kernel over the 64-pixel tiles of jobs[0 .. n) (device array,
// every job of one key), then each job's row kernel over its segments that do not fit a
// wave (jobs_host: the same jobs on the host).
hipError_t composite_jobs_launch(const CompositeJob* jobs, const CompositeJob* jobs_host, int n, const CompositeKey& key,
                                 hipStream_t s);

// Bytes of the coefficient table lf_composite keeps in its context for K planes, V views.
size_t composite_table_bytes(int K, int n_views);
// Fills a's view groups, then launches the composite of a's views.
hipError_t composite_launch(CompositeArgs& a, void* table, hipStream_t s, Profiler* prof = nullptr);
// Validated composite arguments (host); shared by lf_composite and the batch entry points.
lf_status composite_args(const lf_mpi* mpi, const lf_camera* cam, const lf_view* views, int32_t n_views,
                         CompositeArgs* a);
hipError_t plane_coeffs_launch(const CompositeArgs& a, float* bx, float* by, float* cx, float* cy,
                               float* cxn, float* cyn, hipStream_t s);
// Groups the views of `a` for the row kernels (views that share dy, runs of at most G);
// returns a.n_groups.
int view_groups(CompositeArgs& a, int G);
// Pixel rays of the views for SH colour: view v's principal point is (c_x + dx kx, c_y + dy ky)
// (Eq. 5), its rays ((x - c_x,v) / f_x, (y - c_y,v) / f_y, 1) in base-camera axes.
struct ShView {
  float kx, ky, inv_fx, inv_fy;
};
// Composite of SH planes of n_coef coefficients (a.planes float32 texels of
// sh_texel_floats(n_coef)) into a.out (float32 views).
hipError_t composite_sh_launch(CompositeArgs& a, int n_coef, const ShView& sv, hipStream_t s);
// Colour of n Gaussians seen from the world point `centre`.
hipError_t sh_colours_launch(const float* means, const float* sh, int n_coef, int64_t n, const float centre[3],
                             float* rgb, hipStream_t s);
// Zero-fills d_planes [K][hp][wp][4] and accumulates the composite's VJP of d_out into it
// (table: composite_table_bytes(K, V) of device scratch for the sampling coefficients).
hipError_t composite_backward_launch(CompositeArgs& a, void* table, const float* d_out, float* d_planes,
                                    hipStream_t s, Profiler* prof = nullptr);

}  // namespace lf
