// Two D2Q9 BGK steps per launch (temporal blocking through LDS) for gfx950.
//
// A workgroup owns a strip of W columns and a band of H rows of the output
// and marches down its band one row per iteration.  Iteration k computes the
// first step (t -> t+1) on row y0 + k for the W strip columns plus one halo
// column on each side, exactly as the single-step kernel does (pull from
// x - c_l, collide with Eq. 1 / Eq. 2 and Guo forcing).  The six populations
// with c_x != 0 are exchanged between neighbouring columns through a
// double-buffered LDS row; the three with c_x = 0 stay in the thread's
// registers.  The second step (t+1 -> t+2) then updates row y0 + k - 1 from
// rows k - 2 .. k of the first step's output, held in registers, and writes it
// to the destination buffer.  The intermediate state never leaves the CU, so
// two lattice updates cost one read and one write of every population (plus
// one read of the force field): 80 B per site per launch in FP32 instead of
// 2 x 80 B.  Results are bit-identical to two single-step launches (same
// per-site arithmetic, same operand order).
#include <hip/hip_runtime.h>

#include "lbm_internal.h"
#include "lbm_site.h"

namespace lbm {
namespace {

using namespace step_detail;

template <typename T, bool NT>
__device__ __forceinline__ void put(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Threads [0, W) own the strip columns, thread W the left halo column and
// thread W + 1 the right one; blockDim.x = W + 64.  With PF the next row's
// loads are issued before the current row is collided.
template <typename T, bool FORCE, bool NT, bool PF>
__global__ void __launch_bounds__(1024) k_step_fused2(StepParams p, int W, int H, int strips,
                                                      int total, int per_xcd) {
  extern __shared__ unsigned char smem_raw[];
  T* const lds = reinterpret_cast<T*>(smem_raw);
  const int stride = W + 2;
  const int b = blockIdx.x;
  const int tile = (b & 7) * per_xcd + (b >> 3);
  if (tile >= total) return;  // uniform over the workgroup
  const int nx = p.nx, ny = p.ny;
  const int x0 = (tile % strips) * W;
  const int y0 = (tile / strips) * H;
  const int weff = min(W, nx - x0);
  const int heff = min(H, ny - y0);
  const int t = threadIdx.x;
  int col = 0, li = 0;
  bool s1 = false, s2 = false;
  if (t < weff) {
    col = x0 + t;
    li = t + 1;
    s1 = s2 = true;
  } else if (t == W) {
    col = x0 == 0 ? nx - 1 : x0 - 1;
    li = 0;
    s1 = true;
  } else if (t == W + 1) {
    col = x0 + weff == nx ? 0 : x0 + weff;
    li = weff + 1;
    s1 = true;
  }
  const T* __restrict__ src = static_cast<const T*>(p.src);
  T* __restrict__ dst = static_cast<T*>(p.dst);
  const T* __restrict__ gfx = static_cast<const T*>(p.fx);
  const T* __restrict__ gfy = static_cast<const T*>(p.fy);
  const T omega = T(p.omega);
  const T guo = T(1) - T(0.5) * T(p.omega);
  const T alpha = T(p.alpha);

  // first-step output at this column, carried over rows: l = 0 and the
  // x-shifted l = 1, 3 of row r-1; l = 2 and the shifted l = 5, 6 of rows
  // r-1 (a) and r-2 (b); the force of row r-1
  T c0 = T(0), c1 = T(0), c3 = T(0);
  T c2a = T(0), c2b = T(0), c5a = T(0), c5b = T(0), c6a = T(0), c6b = T(0);
  T fxp = T(0), fyp = T(0);

  auto wrap_row = [ny](int r) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); };
  auto load_row = [&](int r, T (&d)[9][1], T& fx, T& fy) {
    const int rn = r == 0 ? ny - 1 : r - 1;
    const int rp = r == ny - 1 ? 0 : r + 1;
    pull_all<T, 1>(src, p.ps, p.rs, nx, col, r, rn, rp, d);
    if constexpr (FORCE) {
      if (gfx) {
        const size_t i = static_cast<size_t>(r) * nx + col;
        fx = gfx[i];
        fy = gfy[i];
      } else {
        fx = fy = T(0);
      }
    }
  };

  T dn[9][1];
  T fxn = T(0), fyn = T(0);
  if constexpr (PF) {
    if (s1) load_row(wrap_row(y0 - 1), dn, fxn, fyn);
  }
  for (int k = -1; k <= heff; ++k) {
    const int r = wrap_row(y0 + k);
    T* const slot = lds + ((k + 1) & 1) * 6 * stride;
    T o[9];
    T fx = T(0), fy = T(0);
    if (s1) {
      T d[9][1];
      if constexpr (PF) {
#pragma unroll
        for (int l = 0; l < 9; ++l) d[l][0] = dn[l][0];
        fx = fxn;
        fy = fyn;
        if (k < heff) load_row(wrap_row(y0 + k + 1), dn, fxn, fyn);
      } else {
        load_row(r, d, fx, fy);
      }
      T di[9];
#pragma unroll
      for (int l = 0; l < 9; ++l) di[l] = d[l][0];
      SiteMoments<T, FORCE> m(di, FORCE ? fx : T(0), FORCE ? fy : T(0), alpha);
      collide_site<T, FORCE>(di, m, omega, guo, o);
      slot[0 * stride + li] = o[1];
      slot[1 * stride + li] = o[3];
      slot[2 * stride + li] = o[5];
      slot[3 * stride + li] = o[6];
      slot[4 * stride + li] = o[7];
      slot[5 * stride + li] = o[8];
    }
    __syncthreads();
    if (s2) {
      // populations that reach this column from its x-neighbours
      const T n1 = slot[0 * stride + li - 1];
      const T n3 = slot[1 * stride + li + 1];
      const T n5 = slot[2 * stride + li - 1];
      const T n6 = slot[3 * stride + li + 1];
      const T n7 = slot[4 * stride + li + 1];
      const T n8 = slot[5 * stride + li - 1];
      if (k >= 1) {
        // second step at (col, y0 + k - 1): d_l = g_l(x - c_l) of the first step
        const T d2[9] = {c0, c1, c2b, c3, o[4], c5b, c6b, n7, n8};
        SiteMoments<T, FORCE> m(d2, FORCE ? fxp : T(0), FORCE ? fyp : T(0), alpha);
        T q[9];
        collide_site<T, FORCE>(d2, m, omega, guo, q);
        T* const out = dst + static_cast<size_t>(y0 + k - 1) * p.rs + col;
#pragma unroll
        for (int l = 0; l < 9; ++l) put<T, NT>(out + l * p.ps, q[l]);
      }
      c0 = o[0];
      c1 = n1;
      c3 = n3;
      c2b = c2a;
      c2a = o[2];
      c5b = c5a;
      c5a = n5;
      c6b = c6a;
      c6a = n6;
      fxp = fx;
      fyp = fy;
    }
  }
}

template <typename T, bool FORCE, bool NT, bool PF>
int launch_t(const StepParams& p, const lbm_tile& t, hipStream_t s) {
  const int W = t.bx, H = t.ry;
  const int strips = (p.nx + W - 1) / W;
  const int bands = (p.ny + H - 1) / H;
  const int total = strips * bands;
  const int per_xcd = (total + 7) / 8;
  const size_t lds = static_cast<size_t>(2) * 6 * (W + 2) * sizeof(T);
  hipLaunchKernelGGL((k_step_fused2<T, FORCE, NT, PF>), dim3(per_xcd * 8), dim3(W + 64), lds, s, p, W,
                     H, strips, total, per_xcd);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <typename T, bool FORCE>
int dispatch(const StepParams& p, const lbm_tile& t, hipStream_t s) {
  if (t.nt) return t.pf ? launch_t<T, FORCE, true, true>(p, t, s) : launch_t<T, FORCE, true, false>(p, t, s);
  return t.pf ? launch_t<T, FORCE, false, true>(p, t, s) : launch_t<T, FORCE, false, false>(p, t, s);
}

}  // namespace

bool fused_tile_ok(const lbm_tile& t, int dtype) {
  if (t.fuse != 2 || t.by != 1 || t.vx != 1) return false;
  if (t.bx < 64 || t.bx % 64 != 0 || t.bx + 64 > 1024) return false;
  if (t.ry < 1 || t.ry > 4096) return false;
  if ((t.nt != 0 && t.nt != 1) || (t.pf != 0 && t.pf != 1)) return false;
  const size_t lds = static_cast<size_t>(2) * 6 * (t.bx + 2) * (dtype == LBM_F64 ? 8 : 4);
  return lds <= 64 * 1024;
}

int launch_step_fused2(int dtype, bool force, const StepParams& p, const lbm_tile& t, hipStream_t s) {
  if (!fused_tile_ok(t, dtype)) return fail(LBM_E_INVALID, "invalid two-step launch shape");
  if (p.h_rho) return fail(LBM_E_INVALID, "the two-step kernel records no moment history");
  if (dtype == LBM_F64)
    return force ? dispatch<double, true>(p, t, s) : dispatch<double, false>(p, t, s);
  return force ? dispatch<float, true>(p, t, s) : dispatch<float, false>(p, t, s);
}

}  // namespace lbm
