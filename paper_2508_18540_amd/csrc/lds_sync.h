// Work-group barrier that orders LDS only.
#pragma once

#include <hip/hip_runtime.h>

namespace lf {

// __syncthreads() also waits for every outstanding global load, store and atomic of the
// calling wave; where threads only exchange data through LDS, this barrier lets prefetched
// loads and fire-and-forget stores / atomics stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace lf
