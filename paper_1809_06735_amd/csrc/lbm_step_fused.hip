// K = 2..6 D2Q9 BGK steps per launch (temporal blocking through LDS) for
// gfx950: the single-grid kernel over the tiles of lbm_fused.h, launch-shape
// validation and dispatch.  K lattice updates cost one read and one write of
// every population plus one read of the force field (80 B per site per launch
// in FP32), bit-identical to K single-step launches.
#include <hip/hip_runtime.h>

#include "lbm_fused.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

using fused_detail::kFusedMaxThreads;

// Workgroups are numbered so that consecutive tiles fall on the same XCD.
template <typename T, int K, bool FORCE, bool NT, bool PF>
__global__ void __launch_bounds__(kFusedMaxThreads) k_step_fused(StepParams p, int W, int H, int strips,
                                                                 int total, int per_xcd, int packed) {
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int tile = (b & 7) * per_xcd + (b >> 3);
  if (tile >= total) return;  // uniform over the workgroup
  fused_detail::fused_tile<T, K, FORCE, NT, PF>(p, reinterpret_cast<T*>(smem_raw), W, H, strips, tile,
                                                packed != 0);
}

// Either launches the kernel (resident == nullptr) or stores in *resident the
// number of its workgroups that the device holds at once over all CUs.
template <typename T, int K, bool FORCE, bool NT, bool PF>
int launch_t(const StepParams& p, const lbm_tile& t, hipStream_t s, int* resident) {
  const int W = fused_strip_width(t), H = t.ry;
  const int threads = t.halo ? t.bx : t.bx + 64;
  const size_t lds = fused_lds_bytes(W, K, sizeof(T) == 8 ? LBM_F64 : LBM_F32);
  if (resident) {
    int per_cu = 0, dev = 0, cus = 0;
    LBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_fused<T, K, FORCE, NT, PF>,
                                                         threads, lds));
    LBM_HIP(hipGetDevice(&dev));
    LBM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    *resident = per_cu * cus;
    return LBM_OK;
  }
  const int strips = (p.nx + W - 1) / W;
  const int bands = (p.ny + H - 1) / H;
  const int total = strips * bands;
  const int per_xcd = (total + 7) / 8;
  hipLaunchKernelGGL((k_step_fused<T, K, FORCE, NT, PF>), dim3(per_xcd * 8), dim3(threads), lds, s, p,
                     W, H, strips, total, per_xcd, t.halo);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <typename T, int K, bool FORCE>
int dispatch_k(const StepParams& p, const lbm_tile& t, hipStream_t s, int* r) {
  if (t.nt)
    return t.pf ? launch_t<T, K, FORCE, true, true>(p, t, s, r) : launch_t<T, K, FORCE, true, false>(p, t, s, r);
  return t.pf ? launch_t<T, K, FORCE, false, true>(p, t, s, r) : launch_t<T, K, FORCE, false, false>(p, t, s, r);
}

template <typename T, bool FORCE>
int dispatch(const StepParams& p, const lbm_tile& t, hipStream_t s, int* r) {
  switch (t.fuse) {
    case 2: return dispatch_k<T, 2, FORCE>(p, t, s, r);
    case 3: return dispatch_k<T, 3, FORCE>(p, t, s, r);
    case 4: return dispatch_k<T, 4, FORCE>(p, t, s, r);
    case 5: return dispatch_k<T, 5, FORCE>(p, t, s, r);
    default: return dispatch_k<T, 6, FORCE>(p, t, s, r);
  }
}

int dispatch_dtype(int dtype, bool force, const StepParams& p, const lbm_tile& t, hipStream_t s, int* r) {
  if (dtype == LBM_F64) return force ? dispatch<double, true>(p, t, s, r) : dispatch<double, false>(p, t, s, r);
  return force ? dispatch<float, true>(p, t, s, r) : dispatch<float, false>(p, t, s, r);
}

}  // namespace

int launch_step_fused(int dtype, bool force, const StepParams& p, const lbm_tile& t, hipStream_t s) {
  if (!fused_tile_ok(t, dtype)) return fail(LBM_E_INVALID, "invalid multi-step launch shape");
  if (p.h_rho) return fail(LBM_E_INVALID, "the multi-step kernel records no moment history");
  return dispatch_dtype(dtype, force, p, t, s, nullptr);
}

int fused_resident_groups(int dtype, bool force, const lbm_tile& t, int* groups) {
  *groups = 0;
  if (!fused_tile_ok(t, dtype)) return fail(LBM_E_INVALID, "invalid multi-step launch shape");
  return dispatch_dtype(dtype, force, StepParams{}, t, nullptr, groups);
}

}  // namespace lbm
