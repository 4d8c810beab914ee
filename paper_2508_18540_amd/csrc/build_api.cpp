// MPI build entry points (Alg. 1 steps 1-5).
#include "lf_internal.h"

using namespace lf;

extern "C" lf_status lf_build_mpi_workspace(const lf_field*, const lf_camera*, int32_t, int64_t, size_t*) {
  return fail(LF_ERR_UNSUPPORTED, "lf_build_mpi_workspace is not available yet");
}

extern "C" lf_status lf_build_mpi(lf_ctx*, const lf_field*, const lf_camera*, int32_t, int32_t, const float*,
                                  lf_mpi*, void*, size_t, void*) {
  return fail(LF_ERR_UNSUPPORTED, "lf_build_mpi is not available yet");
}

extern "C" lf_status lf_build_stats(lf_ctx*, const void*, size_t, lf_build_info*, void*) {
  return fail(LF_ERR_UNSUPPORTED, "lf_build_stats is not available yet");
}
