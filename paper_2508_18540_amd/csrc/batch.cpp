// Batched rendering of several scenes.  Two forms:
//  * streams: each scene's whole build and composite on a stream of its own, forked from
//    and joined back into the caller's stream;
//  * work list (LF_BATCH_WORKLIST): each scene's cull, sort, chunks and tile lists on its
//    own stream, then one splat launch and one merge launch over the work items of every
//    scene (per plane dtype), and one composite launch over the row tiles of every scene
//    (per kernel key), each phase's kernel walking a (scene, item) list.
// Optional capture of the whole batch into one HIP graph, and a composite autotuner that
// picks the view-group size and row-tile width of every scene by timing the candidates
// (cached per process by scene shape).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "build_internal.h"
#include "lf_internal.h"
#include "sort_internal.h"

namespace {

constexpr int kMaxStreams = 16;
constexpr int kGroups[4] = {4, 8, 12, 16};
constexpr int kTiles[2] = {64, 256};

// Tuned (group, tile) per scene shape: camera, plane count and dtype, views, sampling, output.
std::mutex tune_mu;
std::map<std::vector<uint32_t>, std::pair<int, int>> tune_cache;

}  // namespace

struct lf_batch {
  lf_ctx* ctx = nullptr;
  int flags = 0;
  std::vector<lf_batch_item> items;
  std::vector<std::vector<lf_view>> views;
  std::vector<void*> tables;            // per scene composite coefficient table
  std::vector<int> group;               // per scene view-group size (0: default)
  std::vector<int> tile;                // per scene row-tile width (0: default)
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
  hipStream_t cap = nullptr;            // stream the graph is captured on and launched from
  hipEvent_t cap_in = nullptr, cap_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // work list: splat groups (scenes of one plane dtype) with their build arguments at
  // offsets of the device array `dargs`, composite groups (scenes of one kernel key) with
  // their jobs at offsets of `djobs`, and per scene its roles
  void* dev = nullptr;
  lf::BuildArgs* dargs = nullptr;
  lf::CompositeJob* djobs = nullptr;
  std::vector<std::vector<int>> splat_scenes;
  std::vector<int> splat_dtype;
  std::vector<size_t> splat_off;
  std::vector<lf::SplatJobs> splat_jobs;
  std::vector<std::vector<lf::BuildArgs>> dargs_host;
  std::vector<std::vector<int>> comp_scenes;
  std::vector<lf::CompositeKey> comp_keys;
  std::vector<std::vector<lf::CompositeJob>> comp_jobs;
  std::vector<size_t> comp_off;
  std::vector<char> in_splat, in_comp;
};

using namespace lf;

namespace {

void release(lf_batch* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->dev) hipFree(b->dev);
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
  a->tile = b->tile[(size_t)i];
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

bool splat_mergeable(const lf_batch_item& it) { return it.field.kind == LF_GAUSSIANS && it.field.n > 0; }

// The work-list form of one run on stream s (see the file comment).  Scenes outside the
// merged splat (voxel fields, empty fields) build completely on their streams; scenes
// outside the merged composite (per-pixel kernel, 256-pixel row tiles) composite alone
// on s after the merged splat.
lf_status enqueue_worklist(lf_batch* b, hipStream_t s) {
  hipError_t e = hipEventRecord(b->fork, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  const int ns = (int)b->streams.size(), n = (int)b->items.size();
  std::vector<CompositeArgs> solo;                          // scenes that composite alone
  std::vector<int> solo_i;
  for (int i = 0; i < n; ++i) {
    hipStream_t si = b->streams[(size_t)(i % ns)];
    if (i < ns && (e = hipStreamWaitEvent(si, b->fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    lf_batch_item& it = b->items[(size_t)i];
    BuildArgs a;
    BuildLayout L;
    lf_status st = build_prepare(b->ctx, &it.field, &it.cam, it.n_chunk, it.binning,
                                 it.binning == LF_BIN_INV_DEPTH ? it.inv_depth_range : nullptr, &it.mpi, nullptr, 0,
                                 it.workspace, it.workspace_bytes, si, &a, &L);
    if (st != LF_OK) return st;
    bool complete = false;
    if ((e = build_lists(a, L, si, nullptr, &complete)) != hipSuccess) return hip_fail(e, "batch build launch");
    if (!b->in_splat[(size_t)i] && !complete && (e = build_splat(a, L, si, nullptr)) != hipSuccess)
      return hip_fail(e, "batch build launch");
    if (b->in_comp[(size_t)i]) continue;                   // its table is filled below
    CompositeArgs* ca = new (std::nothrow) CompositeArgs;
    if (!ca) return fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
    st = composite_of(b, i, ca);
    if (st == LF_OK && !b->in_splat[(size_t)i]) {
      // complete on its own stream
      e = composite_launch(*ca, b->tables[(size_t)i], si, nullptr);
      if (e != hipSuccess) st = hip_fail(e, "batch composite launch");
    } else if (st == LF_OK) {
      solo.push_back(*ca);
      solo_i.push_back(i);
    }
    delete ca;
    if (st != LF_OK) return st;
  }
  for (size_t g = 0; g < b->comp_scenes.size(); ++g)
    for (size_t q = 0; q < b->comp_scenes[g].size(); ++q) {
      const int i = b->comp_scenes[g][q];
      if ((e = composite_job_table(b->comp_jobs[g][q], b->streams[(size_t)(i % ns)])) != hipSuccess)
        return hip_fail(e, "batch table launch");
    }
  for (int j = 0; j < ns; ++j) {
    if ((e = hipEventRecord(b->done[(size_t)j], b->streams[(size_t)j])) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(s, b->done[(size_t)j], 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  for (size_t g = 0; g < b->splat_scenes.size(); ++g)
    if ((e = splat_batch_launch(b->dargs + b->splat_off[g], b->splat_jobs[g], b->splat_dtype[g], s)) != hipSuccess)
      return hip_fail(e, "batch splat launch");
  for (size_t g = 0; g < b->comp_scenes.size(); ++g)
    if ((e = composite_jobs_launch(b->djobs + b->comp_off[g], b->comp_jobs[g].data(), (int)b->comp_jobs[g].size(),
                                   b->comp_keys[g], s)) != hipSuccess)
      return hip_fail(e, "batch composite launch");
  for (size_t q = 0; q < solo.size(); ++q)
    if ((e = composite_launch(solo[q], b->tables[(size_t)solo_i[q]], s, nullptr)) != hipSuccess)
      return hip_fail(e, "batch composite launch");
  return LF_OK;
}

// Groups the scenes of a work-list batch (by plane dtype for the splat, by kernel key for
// the composite) and uploads their build arguments and composite jobs to device memory.
// Synchronises the device.
lf_status plan_worklist(lf_batch* b) {
  const int n = (int)b->items.size();
  b->in_splat.assign((size_t)n, 0);
  b->in_comp.assign((size_t)n, 0);
  std::vector<BuildArgs> args;
  std::vector<CompositeJob> jobs;
  hipStream_t s0 = b->streams[0];
  for (int i = 0; i < n; ++i) {
    lf_batch_item& it = b->items[(size_t)i];
    if (!splat_mergeable(it)) continue;
    BuildArgs a;
    BuildLayout L;
    lf_status st = build_prepare(b->ctx, &it.field, &it.cam, it.n_chunk, it.binning,
                                 it.binning == LF_BIN_INV_DEPTH ? it.inv_depth_range : nullptr, &it.mpi, nullptr, 0,
                                 it.workspace, it.workspace_bytes, s0, &a, &L);
    if (st != LF_OK) return st;
    // the lists end on the array the tile sort's last pass wrote
    if (radix_passes(L.tile_bits, tile_digit_bits()) & 1) a.evals = a.evals_alt;
    size_t g = 0;
    while (g < b->splat_dtype.size() && b->splat_dtype[g] != it.mpi.dtype) ++g;
    if (g == b->splat_dtype.size()) {
      b->splat_dtype.push_back(it.mpi.dtype);
      b->splat_scenes.emplace_back();
      b->dargs_host.emplace_back();
      SplatJobs none;
      std::memset(&none, 0, sizeof(none));
      none.item_shift = splat_item_shift();
      b->splat_jobs.push_back(none);
    }
    SplatJobs& jb = b->splat_jobs[g];
    jb.n_buckets[jb.n] = L.n_buckets;
    jb.max_items[jb.n] = L.max_items;
    ++jb.n;
    b->splat_scenes[g].push_back(i);
    b->dargs_host[g].push_back(a);
    b->in_splat[(size_t)i] = 1;
  }
  for (int i = 0; i < n; ++i) {
    if (!b->in_splat[(size_t)i]) continue;
    CompositeArgs* ca = new (std::nothrow) CompositeArgs;
    if (!ca) return fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
    lf_status st = composite_of(b, i, ca);
    CompositeJob* j = st == LF_OK ? new (std::nothrow) CompositeJob : nullptr;
    if (st == LF_OK && !j) st = fail(LF_ERR_OUT_OF_MEMORY, "argument block allocation failed");
    CompositeKey key;
    if (st == LF_OK && composite_job(*ca, b->tables[(size_t)i], j, &key)) {
      size_t g = 0;
      while (g < b->comp_keys.size() && !(b->comp_keys[g] == key)) ++g;
      if (g == b->comp_keys.size()) {
        b->comp_keys.push_back(key);
        b->comp_scenes.emplace_back();
        b->comp_jobs.emplace_back();
      }
      b->comp_scenes[g].push_back(i);
      b->comp_jobs[g].push_back(*j);
      b->in_comp[(size_t)i] = 1;
    }
    delete j;
    delete ca;
    if (st != LF_OK) return st;
  }
  size_t na = 0, nj = 0;
  for (auto& v : b->dargs_host) {
    b->splat_off.push_back(na);
    na += v.size();
  }
  for (auto& v : b->comp_jobs) {
    b->comp_off.push_back(nj);
    nj += v.size();
  }
  const size_t bytes_a = ((na * sizeof(BuildArgs) + 255) / 256) * 256;
  const size_t bytes_j = ((nj * sizeof(CompositeJob) + 255) / 256) * 256;
  const size_t bytes_p = b->splat_jobs.size() * (2 * (size_t)kMaxSplatJobs + 2) * 4;
  hipError_t e = hipMalloc(&b->dev, bytes_a + bytes_j + bytes_p + 256);
  if (e != hipSuccess) return hip_fail(e, "batch work list allocation");
  b->dargs = static_cast<BuildArgs*>(b->dev);
  b->djobs = reinterpret_cast<CompositeJob*>(static_cast<char*>(b->dev) + bytes_a);
  uint32_t* pre = reinterpret_cast<uint32_t*>(static_cast<char*>(b->dev) + bytes_a + bytes_j);
  for (size_t g = 0; g < b->splat_jobs.size(); ++g) b->splat_jobs[g].prefix = pre + g * (2 * (size_t)kMaxSplatJobs + 2);
  for (size_t g = 0; g < b->dargs_host.size() && e == hipSuccess; ++g)
    e = hipMemcpy(b->dargs + b->splat_off[g], b->dargs_host[g].data(), b->dargs_host[g].size() * sizeof(BuildArgs),
                  hipMemcpyHostToDevice);
  for (size_t g = 0; g < b->comp_jobs.size() && e == hipSuccess; ++g)
    e = hipMemcpy(b->djobs + b->comp_off[g], b->comp_jobs[g].data(), b->comp_jobs[g].size() * sizeof(CompositeJob),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "batch work list upload");
  return LF_OK;
}

// Tuning key of scene i: its camera, plane count and dtype, views, sampling and output dtype.
std::vector<uint32_t> tune_key(const lf_batch* b, int i) {
  const lf_batch_item& it = b->items[(size_t)i];
  std::vector<uint32_t> k(sizeof(lf_camera) / 4);
  std::memcpy(k.data(), &it.cam, sizeof(lf_camera));
  for (int32_t v : {it.n_chunk, it.mpi.dtype, it.interp, it.out_dtype, it.n_views}) k.push_back((uint32_t)v);
  const size_t o = k.size();
  k.resize(o + 2 * (size_t)it.n_views);
  std::memcpy(k.data() + o, b->views[(size_t)i].data(), sizeof(lf_view) * (size_t)it.n_views);
  return k;
}

// Times every (view-group size, row-tile width) on scene i's planes (built first) and keeps
// the fastest; a scene of a shape tuned before in this process takes the cached choice.
lf_status autotune_scene(lf_batch* b, int i) {
  const std::vector<uint32_t> key = tune_key(b, i);
  {
    std::lock_guard<std::mutex> lk(tune_mu);
    auto f = tune_cache.find(key);
    if (f != tune_cache.end()) {
      b->group[(size_t)i] = f->second.first;
      b->tile[(size_t)i] = f->second.second;
      return LF_OK;
    }
  }
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
  int best_g = 0, best_t = 64;
  for (int c = 0; st == LF_OK && e == hipSuccess && c < 8; ++c) {
    a->group = kGroups[c % 4];
    a->tile = kTiles[c / 4];
    e = composite_launch(*a, b->tables[(size_t)i], s, nullptr);               // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = composite_launch(*a, b->tables[(size_t)i], s, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms < best) {
      best = ms;
      best_g = kGroups[c % 4];
      best_t = kTiles[c / 4];
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  delete a;
  if (st != LF_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "composite autotune");
  b->group[(size_t)i] = best_g;
  b->tile[(size_t)i] = best_t;
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_cache[key] = std::make_pair(best_g, best_t);
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
  if (flags & ~(LF_BATCH_GRAPH | LF_BATCH_AUTOTUNE | LF_BATCH_WORKLIST))
    return fail(LF_ERR_INVALID_ARG, "unknown batch flags 0x%x", flags);
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
  b->tile.assign((size_t)n_items, 0);
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
  if (flags & LF_BATCH_WORKLIST) {
    lf_status st = plan_worklist(b);
    if (st != LF_OK) {
      release(b);
      return st;
    }
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
  auto enqueue = [&](hipStream_t q) { return (b->flags & LF_BATCH_WORKLIST) ? enqueue_worklist(b, q) : enqueue_all(b, q); };
  if (!(b->flags & LF_BATCH_GRAPH)) {
    st = enqueue(s);
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
      st = enqueue(c);
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

extern "C" lf_status lf_batch_tile(const lf_batch* b, int32_t item, int32_t* tile) {
  if (!b || !tile) return fail(LF_ERR_INVALID_ARG, "batch or tile is NULL");
  if (item < 0 || item >= (int32_t)b->items.size()) return fail(LF_ERR_INVALID_ARG, "item %d out of range", item);
  *tile = b->tile[(size_t)item];
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
