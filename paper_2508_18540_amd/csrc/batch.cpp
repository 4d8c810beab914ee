// Batched rendering of several scenes: per-scene streams forked from the caller's stream,
// optional capture of the whole batch into one HIP graph, and a composite autotuner that
// picks the view-group size of every scene by timing the candidates.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "build_internal.h"
#include "lf_internal.h"

namespace {

constexpr int kMaxStreams = 16;
constexpr int kGroups[4] = {4, 8, 12, 16};

}  // namespace

struct lf_batch {
  lf_ctx* ctx = nullptr;
  int flags = 0;
  std::vector<lf_batch_item> items;
  std::vector<std::vector<lf_view>> views;
  std::vector<void*> tables;            // per scene composite coefficient table
  std::vector<int> group;               // per scene view-group size (0: default)
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
  hipStream_t cap = nullptr;            // stream the graph is captured on and launched from
  hipEvent_t cap_in = nullptr, cap_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

using namespace lf;

namespace {

void release(lf_batch* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (void* t : b->tables)
    if (t) hipFree(t);
  for (hipStream_t s : b->streams)
    if (s) hipStreamDestroy(s);
  for (hipEvent_t e : b->done)
    if (e) hipEventDestroy(e);
  if (b->fork) hipEventDestroy(b->fork);
  if (b->cap_in) hipEventDestroy(b->cap_in);
  if (b->cap_out) hipEventDestroy(b->cap_out);
  if (b->cap) hipStreamDestroy(b->cap);
  delete b;
}

lf_status composite_of(const lf_batch* b, int i, CompositeArgs* a) {
  const lf_batch_item& it = b->items[(size_t)i];
  lf_status s = composite_args(&it.mpi, &it.cam, b->views[(size_t)i].data(), it.n_views, a);
  if (s != LF_OK) return s;
  a->interp = it.interp;
  a->out_dtype = it.out_dtype;
  a->out = it.out;
  a->group = b->group[(size_t)i];
  return LF_OK;
}

// Build and composite of scene i on stream s (no profiling: the batch may be captured).
lf_status enqueue_scene(lf_batch* b, int i, hipStream_t s) {
  lf_batch_item& it = b->items[(size_t)i];
  lf_status st = lf_build_mpi(b->ctx, &it.field, &it.cam, it.n_chunk, it.binning,
                              it.binning == LF_BIN_INV_DEPTH ? it.inv_depth_range : nullptr, &it.mpi, it.workspace,
                              it.workspace_bytes, s);
  if (st != LF_OK) return st;
  CompositeArgs* a = new (std::nothrow) CompositeArgs;
  if (!a) return fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
  st = composite_of(b, i, a);
  if (st == LF_OK) {
    hipError_t e = composite_launch(*a, b->tables[(size_t)i], s, nullptr);
    if (e != hipSuccess) st = hip_fail(e, "batch composite launch");
  }
  delete a;
  return st;
}

lf_status enqueue_all(lf_batch* b, hipStream_t s) {
  hipError_t e = hipEventRecord(b->fork, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  const int ns = (int)b->streams.size();
  for (int i = 0; i < (int)b->items.size(); ++i) {
    hipStream_t si = b->streams[(size_t)(i % ns)];
    if (i < ns && (e = hipStreamWaitEvent(si, b->fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    lf_status st = enqueue_scene(b, i, si);
    if (st != LF_OK) return st;
  }
  for (int j = 0; j < ns; ++j) {
    if ((e = hipEventRecord(b->done[(size_t)j], b->streams[(size_t)j])) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(s, b->done[(size_t)j], 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  return LF_OK;
}

// Times every view-group size on scene i's planes (built first) and keeps the fastest.
lf_status autotune_scene(lf_batch* b, int i) {
  hipStream_t s = b->streams[0];
  lf_batch_item& it = b->items[(size_t)i];
  lf_status st = lf_build_mpi(b->ctx, &it.field, &it.cam, it.n_chunk, it.binning,
                              it.binning == LF_BIN_INV_DEPTH ? it.inv_depth_range : nullptr, &it.mpi, it.workspace,
                              it.workspace_bytes, s);
  if (st != LF_OK) return st;
  CompositeArgs* a = new (std::nothrow) CompositeArgs;
  if (!a) return fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
  st = composite_of(b, i, a);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  if (st == LF_OK) e = hipEventCreate(&e0);
  if (st == LF_OK && e == hipSuccess) e = hipEventCreate(&e1);
  float best = INFINITY;
  int best_g = 0;
  for (int gi = 0; st == LF_OK && e == hipSuccess && gi < 4; ++gi) {
    a->group = kGroups[gi];
    e = composite_launch(*a, b->tables[(size_t)i], s, nullptr);               // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = composite_launch(*a, b->tables[(size_t)i], s, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms < best) {
      best = ms;
      best_g = kGroups[gi];
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  delete a;
  if (st != LF_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "composite autotune");
  b->group[(size_t)i] = best_g;
  return LF_OK;
}

}  // namespace

extern "C" lf_status lf_batch_create(lf_ctx* ctx, const lf_batch_item* items, int32_t n_items, int32_t flags,
                                     lf_batch** out) {
  if (!out) return fail(LF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(LF_ERR_INVALID_ARG, "ctx is NULL");
  if (!items) return fail(LF_ERR_INVALID_ARG, "items is NULL");
  if (n_items < 1 || n_items > LF_MAX_BATCH)
    return fail(LF_ERR_INVALID_ARG, "n_items %d outside [1, %d]", n_items, LF_MAX_BATCH);
  if (flags & ~(LF_BATCH_GRAPH | LF_BATCH_AUTOTUNE)) return fail(LF_ERR_INVALID_ARG, "unknown batch flags 0x%x", flags);
  // validate every scene on the host before anything is allocated
  for (int i = 0; i < n_items; ++i) {
    const lf_batch_item& it = items[i];
    size_t need = 0;
    lf_status st = lf_build_mpi_workspace(&it.field, &it.cam, it.n_chunk, 0, &need);
    if (st != LF_OK) return st;
    if (it.binning != LF_BIN_QUANTILE && it.binning != LF_BIN_INV_DEPTH)
      return fail(LF_ERR_INVALID_ARG, "item %d: binning %d is not QUANTILE/INV_DEPTH", i, it.binning);
    if (it.interp != LF_NEAREST && it.interp != LF_BILINEAR)
      return fail(LF_ERR_INVALID_ARG, "item %d: interp %d is not NEAREST/BILINEAR", i, it.interp);
    if (it.out_dtype != LF_F32 && it.out_dtype != LF_F16)
      return fail(LF_ERR_INVALID_ARG, "item %d: out_dtype %d is not F32/F16", i, it.out_dtype);
    if (!it.out || !it.workspace) return fail(LF_ERR_INVALID_ARG, "item %d: out or workspace is NULL", i);
    if (it.mpi.n_chunk != it.n_chunk) return fail(LF_ERR_INVALID_ARG, "item %d: mpi n_chunk differs", i);
    CompositeArgs* a = new (std::nothrow) CompositeArgs;
    if (!a) return fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
    st = composite_args(&it.mpi, &it.cam, it.views, it.n_views, a);
    delete a;
    if (st != LF_OK) return st;
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  lf_batch* b = new (std::nothrow) lf_batch;
  if (!b) return fail(LF_ERR_OUT_OF_MEMORY, "batch allocation failed");
  b->ctx = ctx;
  b->flags = flags;
  b->items.assign(items, items + n_items);
  b->views.resize((size_t)n_items);
  b->tables.assign((size_t)n_items, nullptr);
  b->group.assign((size_t)n_items, 0);
  for (int i = 0; i < n_items; ++i) {
    b->views[(size_t)i].assign(items[i].views, items[i].views + items[i].n_views);
    b->items[(size_t)i].views = b->views[(size_t)i].data();
    if (e == hipSuccess) e = hipMalloc(&b->tables[(size_t)i], composite_table_bytes(items[i].n_chunk, items[i].n_views));
  }
  int ns = n_items < kMaxStreams ? n_items : kMaxStreams;
  // LF_BATCH_STREAMS caps the number of scene streams (1 renders the scenes one by one)
  if (const char* env = getenv("LF_BATCH_STREAMS")) {
    const int v = atoi(env);
    if (v >= 1 && v < ns) ns = v;
  }
  b->streams.assign((size_t)ns, nullptr);
  b->done.assign((size_t)ns, nullptr);
  for (int j = 0; j < ns && e == hipSuccess; ++j) {
    e = hipStreamCreateWithFlags(&b->streams[(size_t)j], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done[(size_t)j], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess && (flags & LF_BATCH_GRAPH)) {
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->cap_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->cap_out, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    release(b);
    return hip_fail(e, "batch resources");
  }
  if (flags & LF_BATCH_AUTOTUNE) {
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    for (int i = 0; i < n_items; ++i) {
      lf_status st = autotune_scene(b, i);
      if (st != LF_OK) {
        ctx->prof.on = prof;
        release(b);
        return st;
      }
    }
    ctx->prof.on = prof;
  }
  *out = b;
  return LF_OK;
}

extern "C" lf_status lf_batch_run(lf_batch* b, void* stream) {
  if (!b) return fail(LF_ERR_INVALID_ARG, "batch is NULL");
  hipError_t e = hipSetDevice(b->ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const bool prof = b->ctx->prof.on;
  b->ctx->prof.on = false;                                 // no event records inside the batch
  lf_status st = LF_OK;
  if (!(b->flags & LF_BATCH_GRAPH)) {
    st = enqueue_all(b, s);
  } else {
    // the graph lives on a private stream (the caller's may be the legacy default stream,
    // which cannot be captured), ordered after the caller's work and joined back into it
    hipStream_t c = b->cap;
    if (!b->exec) {
      e = hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        b->ctx->prof.on = prof;
        return hip_fail(e, "hipStreamBeginCapture");
      }
      st = enqueue_all(b, c);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(c, &g);
      if (st == LF_OK && e != hipSuccess) st = hip_fail(e, "hipStreamEndCapture");
      if (st == LF_OK) {
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
      }
      if (st == LF_OK) b->graph = g;
      else if (g) hipGraphDestroy(g);
    }
    if (st == LF_OK) {
      e = hipEventRecord(b->cap_in, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(c, b->cap_in, 0);
      if (e == hipSuccess) e = hipGraphLaunch(b->exec, c);
      if (e == hipSuccess) e = hipEventRecord(b->cap_out, c);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, b->cap_out, 0);
      if (e != hipSuccess) st = hip_fail(e, "batch graph launch");
    }
  }
  b->ctx->prof.on = prof;
  return st;
}

extern "C" lf_status lf_batch_group(const lf_batch* b, int32_t item, int32_t* group) {
  if (!b || !group) return fail(LF_ERR_INVALID_ARG, "batch or group is NULL");
  if (item < 0 || item >= (int32_t)b->items.size()) return fail(LF_ERR_INVALID_ARG, "item %d out of range", item);
  *group = b->group[(size_t)item];
  return LF_OK;
}

extern "C" lf_status lf_batch_stats(lf_batch* b, lf_build_info* out, int32_t* n_failed, void* stream) {
  if (!b) return fail(LF_ERR_INVALID_ARG, "batch is NULL");
  hipError_t e = hipSetDevice(b->ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const size_t n = b->items.size();
  std::vector<BuildHeader> h(n);
  for (size_t i = 0; i < n; ++i) {
    if (b->items[i].workspace_bytes < sizeof(BuildHeader))
      return fail(LF_ERR_INVALID_ARG, "scene %zu: workspace too small", i);
    if ((e = hipMemcpyAsync(&h[i], b->items[i].workspace, sizeof(BuildHeader), hipMemcpyDeviceToHost,
                            (hipStream_t)stream)) != hipSuccess)
      return hip_fail(e, "hipMemcpyAsync");
  }
  if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  int failed = 0, first_stall = -1, first_over = -1;
  for (size_t i = 0; i < n; ++i) {
    if (out) {
      out[i].n_visible = h[i].n_vis;
      out[i].entries_needed = h[i].entries;
      out[i].entry_capacity = h[i].capacity;
      out[i].overflow = h[i].overflow;
      out[i].stalled = h[i].stalled ? 1 : 0;
    }
    if (h[i].stalled && first_stall < 0) first_stall = (int)i;
    if (h[i].overflow && first_over < 0) first_over = (int)i;
    failed += (h[i].stalled || h[i].overflow) ? 1 : 0;
  }
  if (n_failed) *n_failed = failed;
  if (first_stall >= 0)
    return fail(LF_ERR_HIP, "scene %d: a device-wide wait of its build timed out (its planes are invalid); %d "
                "scene(s) failed", first_stall, failed);
  if (first_over >= 0)
    return fail(LF_ERR_CAPACITY, "scene %d: the build needed %lld entries but the workspace holds %lld; %d scene(s) "
                "failed", first_over, (long long)h[(size_t)first_over].entries,
                (long long)h[(size_t)first_over].capacity, failed);
  return LF_OK;
}

extern "C" void lf_batch_destroy(lf_batch* b) { release(b); }
