// D2Q9 BGK step, initialisation, moments and copy kernels for gfx950.
//
// Storage: population l at site (y, x) is element l * ps + y * rs + x (either
// nine planes [9][ny][nx] or nine rows per grid row [ny][9][nx]) and holds
// f_l - w_l (the deviation from the rest state), x fastest.  The state at time t is kept
// "un-streamed": plane l at site y holds f_l(y + c_l, t), so the pre-collision
// populations at x are pulled from x - c_l, and one step is a single pass
// that pulls, collides (Eq. 1 with the equilibrium of Eq. 2) and writes the
// post-collision values back at x into the other buffer.  Every population is
// read once and written once per step: 9 + 9 values per lattice update.
#include <hip/hip_runtime.h>

#include "lbm_internal.h"
#include "lbm_reduce.h"
#include "lbm_site.h"

namespace lbm {
namespace {

using namespace step_detail;
using namespace reduce_detail;

// One step over a tile of (blockDim.x * VX) x (blockDim.y * ry) sites.
// Workgroups are numbered so that consecutive tiles fall on the same XCD
// (the hardware deals workgroups round-robin over the 8 XCDs).
template <typename T, int VX, bool FORCE, bool NT>
__global__ void __launch_bounds__(1024) k_step(StepParams p, int tiles_x, int total, int per_xcd,
                                               int ry) {
  const int b = blockIdx.x;
  const int tile = (b & 7) * per_xcd + (b >> 3);
  if (tile >= total) return;
  const int tx = tile % tiles_x;
  const int ty = tile / tiles_x;
  const int x0 = (tx * blockDim.x + threadIdx.x) * VX;
  if (x0 >= p.nx) return;
  const int ybase = (ty * blockDim.y + threadIdx.y) * ry;
  const int nx = p.nx, ny = p.ny;
  const T* __restrict__ src = static_cast<const T*>(p.src);
  T* __restrict__ dst = static_cast<T*>(p.dst);
  const T omega = T(p.omega);
  const T guo = T(1) - T(0.5) * T(p.omega);
  const T alpha = T(p.alpha);
  for (int k = 0; k < ry; ++k) {
    const int y = ybase + k;
    if (y >= ny) break;
    const int yn = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    T d[9][VX];
    pull_all<T, VX>(src, p.ps, p.rs, nx, x0, y, yn, yp, d);
    const size_t row = static_cast<size_t>(y) * nx + x0;
    T fx[VX], fy[VX];
    if constexpr (FORCE) {
      if (p.fx) {
        load_aligned<T, VX>(static_cast<const T*>(p.fx) + row, fx);
        load_aligned<T, VX>(static_cast<const T*>(p.fy) + row, fy);
      } else {
#pragma unroll
        for (int i = 0; i < VX; ++i) fx[i] = fy[i] = T(0);
      }
    }
    T o[9][VX];
    double hr[VX], hx[VX], hy[VX];
#pragma unroll
    for (int i = 0; i < VX; ++i) {
      T di[9];
#pragma unroll
      for (int l = 0; l < 9; ++l) di[l] = d[l][i];
      SiteMoments<T, FORCE> m(di, FORCE ? fx[i] : T(0), FORCE ? fy[i] : T(0), alpha);
      T oi[9];
      collide_site<T, FORCE>(di, m, omega, guo, oi);
#pragma unroll
      for (int l = 0; l < 9; ++l) o[l][i] = oi[l];
      hr[i] = 1.0 + double(m.drho);  // rho - 1 kept to the storage type's precision
      hx[i] = double(m.ux);
      hy[i] = double(m.uy);
    }
#pragma unroll
    for (int l = 0; l < 9; ++l)
      store_aligned<T, VX, NT>(dst + l * p.ps + static_cast<size_t>(y) * p.rs + x0, o[l]);
    if (p.h_rho) {
#pragma unroll
      for (int i = 0; i < VX; ++i) {
        p.h_rho[row + i] = hr[i];
        p.h_ux[row + i] = hx[i];
        p.h_uy[row + i] = hy[i];
      }
    }
  }
}

// f(x, 0) = f^eq(rho0(x), u0(x)) stored un-streamed: plane l at x - c_l.
template <typename T>
__global__ void __launch_bounds__(256) k_init(T* __restrict__ pop, PopLayout lay,
                                              const double* __restrict__ rho0,
                                              const double* __restrict__ ux0,
                                              const double* __restrict__ uy0, int nx, int ny) {
  const size_t plane = static_cast<size_t>(nx) * ny;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < plane;
       i += size_t(gridDim.x) * blockDim.x) {
    const int x = static_cast<int>(i % nx);
    const int y = static_cast<int>(i / nx);
    const double rho = rho0[i], ux = ux0[i], uy = uy0[i];
    const double usq15 = 1.5 * (ux * ux + uy * uy);
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      const double cu = cxq(l) * ux + cyq(l) * uy;
      const double dev = wq(l) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - usq15));
      int xs = x - cxq(l), ys = y - cyq(l);
      xs += xs < 0 ? nx : 0;
      xs -= xs >= nx ? nx : 0;
      ys += ys < 0 ? ny : 0;
      ys -= ys >= ny ? ny : 0;
      pop[l * lay.ps + static_cast<size_t>(ys) * lay.rs + xs] = T(dev);
    }
  }
}

// ---- moments ------------------------------------------------------------------------
constexpr int kMomThreads = kRedThreads;
constexpr int kMomMaxBlocks = 1024;

template <typename T, typename O, bool FORCE>
__global__ void __launch_bounds__(kMomThreads) k_moments(MomentParams p) {
  const int nx = p.nx, ny = p.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const T* __restrict__ pop = static_cast<const T*>(p.pop);
  const T alpha = T(p.alpha);
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 1.0e300, 0.0};
  for (size_t i = blockIdx.x * size_t(kMomThreads) + threadIdx.x; i < plane;
       i += size_t(gridDim.x) * kMomThreads) {
    const int x = static_cast<int>(i % nx);
    const int y = static_cast<int>(i / nx);
    T d[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      int xs = x - cxq(l), ys = y - cyq(l);
      xs += xs < 0 ? nx : 0;
      xs -= xs >= nx ? nx : 0;
      ys += ys < 0 ? ny : 0;
      ys -= ys >= ny ? ny : 0;
      d[l] = pop[l * p.ps + static_cast<size_t>(ys) * p.rs + xs];
    }
    T fx = T(0), fy = T(0);
    if constexpr (FORCE) {
      if (p.fx) {
        fx = static_cast<const T*>(p.fx)[i];
        fy = static_cast<const T*>(p.fy)[i];
      }
    }
    SiteMoments<T, FORCE> m(d, fx, fy, alpha);
    // rho = 1 + drho formed in FP64: with FP32 storage, 1 + drho in FP32 would round
    // the density variation to the FP32 spacing at 1 (6e-8)
    const double r = 1.0 + double(m.drho), vx = m.ux, vy = m.uy;
    if (p.rho) static_cast<O*>(p.rho)[i] = O(r);
    if (p.ux) static_cast<O*>(p.ux)[i] = O(m.ux);
    if (p.uy) static_cast<O*>(p.uy)[i] = O(m.uy);
    if (p.rho64) {
      p.rho64[i] = r;
      p.ux64[i] = vx;
      p.uy64[i] = vy;
    }
    if (p.ftx64) {
      p.ftx64[i] = double(m.Fx);
      p.fty64[i] = double(m.Fy);
    }
    const double s2 = vx * vx + vy * vy;
    const bool finite = isfinite(r) && isfinite(vx) && isfinite(vy);
    acc[0] += r;
    acc[1] += r * vx;
    acc[2] += r * vy;
    acc[3] += 0.5 * r * s2;
    acc[4] = fmax(acc[4], sqrt(s2));
    acc[5] = fmin(acc[5], r);
    acc[6] += finite ? 0.0 : 1.0;
  }
  block_reduce7(acc, p.partials + blockIdx.x * 8);
}

__global__ void __launch_bounds__(kMomThreads) k_reduce_scalars(const double* __restrict__ part,
                                                                int nblocks, double* out) {
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 1.0e300, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kMomThreads) {
    const double* q = part + b * 8;
    acc[0] += q[0];
    acc[1] += q[1];
    acc[2] += q[2];
    acc[3] += q[3];
    acc[4] = fmax(acc[4], q[4]);
    acc[5] = fmin(acc[5], q[5]);
    acc[6] += q[6];
  }
  block_reduce7(acc, out);
}

template <typename T>
__global__ void k_to_storage(T* __restrict__ dst, const double* __restrict__ src, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x)
    dst[i] = T(src[i]);
}

typedef float f4a __attribute__((ext_vector_type(4), aligned(16)));
constexpr int kCopyUnroll = 4;
// Each workgroup copies 256 * kCopyUnroll 16-byte vectors; all loads of a
// thread are issued before its stores.
__global__ void __launch_bounds__(256) k_copy(f4a* __restrict__ dst, const f4a* __restrict__ src,
                                              size_t n) {
  const size_t base = blockIdx.x * size_t(256 * kCopyUnroll) + threadIdx.x;
  f4a v[kCopyUnroll];
#pragma unroll
  for (int k = 0; k < kCopyUnroll; ++k) {
    const size_t i = base + size_t(k) * 256;
    if (i < n) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < kCopyUnroll; ++k) {
    const size_t i = base + size_t(k) * 256;
    if (i < n) __builtin_nontemporal_store(v[k], dst + i);
  }
}

int grid_for(size_t n, int threads, int cap) {
  size_t b = (n + threads - 1) / threads;
  if (b > static_cast<size_t>(cap)) b = cap;
  if (b < 1) b = 1;
  return static_cast<int>(b);
}

template <typename T, int VX, bool FORCE, bool NT>
int launch_step_t(const StepParams& p, const lbm_tile& t, hipStream_t s) {
  const int tiles_x = (p.nx / VX + t.bx - 1) / t.bx;
  const int rows_per_tile = t.by * t.ry;
  const int tiles_y = (p.ny + rows_per_tile - 1) / rows_per_tile;
  const int total = tiles_x * tiles_y;
  const int per_xcd = (total + 7) / 8;
  dim3 block(t.bx, t.by);
  hipLaunchKernelGGL((k_step<T, VX, FORCE, NT>), dim3(per_xcd * 8), block, 0, s, p, tiles_x, total,
                     per_xcd, t.ry);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <typename T, bool FORCE, bool NT>
int dispatch_vx(const StepParams& p, const lbm_tile& t, hipStream_t s) {
  switch (t.vx) {
    case 1: return launch_step_t<T, 1, FORCE, NT>(p, t, s);
    case 2: return launch_step_t<T, 2, FORCE, NT>(p, t, s);
    case 4: return launch_step_t<T, 4, FORCE, NT>(p, t, s);
    default: return fail(LBM_E_INVALID, "tile vx must be 1, 2 or 4 (got %d)", t.vx);
  }
}

template <typename T>
int dispatch_step(bool force, const StepParams& p, const lbm_tile& t, hipStream_t s) {
  if (force) return t.nt ? dispatch_vx<T, true, true>(p, t, s) : dispatch_vx<T, true, false>(p, t, s);
  return t.nt ? dispatch_vx<T, false, true>(p, t, s) : dispatch_vx<T, false, false>(p, t, s);
}

}  // namespace

int launch_step(int dtype, bool force, const StepParams& p, const lbm_tile& t, hipStream_t s) {
  if (t.fuse >= 2) return launch_step_fused(dtype, force, p, t, s);
  if (dtype == LBM_F32) return dispatch_step<float>(force, p, t, s);
  return dispatch_step<double>(force, p, t, s);
}

int launch_init(int dtype, void* pop, PopLayout lay, const double* rho0, const double* ux0,
                const double* uy0, int nx, int ny, hipStream_t s) {
  const size_t n = static_cast<size_t>(nx) * ny;
  const int g = grid_for(n, 256, 4096);
  if (dtype == LBM_F32)
    hipLaunchKernelGGL(k_init<float>, dim3(g), dim3(256), 0, s, static_cast<float*>(pop), lay, rho0,
                       ux0, uy0, nx, ny);
  else
    hipLaunchKernelGGL(k_init<double>, dim3(g), dim3(256), 0, s, static_cast<double*>(pop), lay,
                       rho0, ux0, uy0, nx, ny);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

int moment_blocks(int nx, int ny) {
  return grid_for(static_cast<size_t>(nx) * ny, kMomThreads, kMomMaxBlocks);
}

template <typename T, bool FORCE>
static int launch_moments_t(const MomentParams& p, hipStream_t s) {
  const int g = moment_blocks(p.nx, p.ny);
  if (p.out_dtype == LBM_F32)
    hipLaunchKernelGGL((k_moments<T, float, FORCE>), dim3(g), dim3(kMomThreads), 0, s, p);
  else
    hipLaunchKernelGGL((k_moments<T, double, FORCE>), dim3(g), dim3(kMomThreads), 0, s, p);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

int launch_moments(int dtype, bool force, const MomentParams& p, hipStream_t s) {
  if (dtype == LBM_F32)
    return force ? launch_moments_t<float, true>(p, s) : launch_moments_t<float, false>(p, s);
  return force ? launch_moments_t<double, true>(p, s) : launch_moments_t<double, false>(p, s);
}

int launch_reduce_scalars(const double* partials, int nblocks, double* out8, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_scalars, dim3(1), dim3(kMomThreads), 0, s, partials, nblocks, out8);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

int launch_to_storage(int dtype, void* dst, const double* src, size_t n, hipStream_t s) {
  const int g = grid_for(n, 256, 4096);
  if (dtype == LBM_F32)
    hipLaunchKernelGGL(k_to_storage<float>, dim3(g), dim3(256), 0, s, static_cast<float*>(dst), src,
                       n);
  else
    hipLaunchKernelGGL(k_to_storage<double>, dim3(g), dim3(256), 0, s, static_cast<double*>(dst),
                       src, n);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

int launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 16;
  const size_t per = size_t(256) * kCopyUnroll;
  if ((n + per - 1) / per > 0x7fffffffu) return fail(LBM_E_INVALID, "copy too large");
  const int g = static_cast<int>((n + per - 1) / per);
  hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, s, static_cast<f4a*>(dst),
                     static_cast<const f4a*>(src), n);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

}  // namespace lbm
