// Batched ensemble (filled in below).
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

using namespace lbm;

extern "C" {
int lbm_batch_workspace_bytes(const lbm_config*, int32_t, size_t*) { return fail(LBM_E_UNSUPPORTED, "batch: not built"); }
int lbm_batch_init(const lbm_config*, int32_t, void*, size_t, const double* const*, const double* const*,
                   const double* const*, const double* const*, const double* const*, lbm_batch*) {
  return fail(LBM_E_UNSUPPORTED, "batch: not built");
}
int lbm_batch_set_mode(lbm_batch, int32_t, int32_t) { return fail(LBM_E_UNSUPPORTED, "batch: not built"); }
int lbm_batch_set_tile(lbm_batch, int32_t, int32_t, int32_t) { return fail(LBM_E_UNSUPPORTED, "batch: not built"); }
int lbm_batch_autotune(lbm_batch, int32_t, int32_t*, int32_t*, int32_t*) { return fail(LBM_E_UNSUPPORTED, "batch: not built"); }
int lbm_batch_step(lbm_batch, int64_t) { return fail(LBM_E_UNSUPPORTED, "batch: not built"); }
int lbm_batch_moments(lbm_batch, int32_t, void*, void*, void*, int32_t, double*) { return fail(LBM_E_UNSUPPORTED, "batch: not built"); }
int lbm_batch_time(lbm_batch, int64_t*) { return fail(LBM_E_UNSUPPORTED, "batch: not built"); }
int64_t lbm_batch_sites(lbm_batch) { return 0; }
int lbm_batch_destroy(lbm_batch) { return LBM_OK; }
}
