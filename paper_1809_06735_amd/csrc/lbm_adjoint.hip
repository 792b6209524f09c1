// Discrete adjoint (filled in below).
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

using namespace lbm;

extern "C" {
int lbm_adjoint_workspace_bytes(const lbm_adjoint_config*, size_t*) { return fail(LBM_E_UNSUPPORTED, "adjoint: not built"); }
int lbm_adjoint_run(const lbm_adjoint_config*, void*, size_t, const double*, const double*, double*, double*,
                    double*, double*) {
  return fail(LBM_E_UNSUPPORTED, "adjoint: not built");
}
}
