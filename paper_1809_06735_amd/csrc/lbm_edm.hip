// The paper's own forcing (Sec. 3, Eqs. 14-16) for gfx950: Kupershtokh's
// exact-difference method with a static external force plus the spectral
// damping of the large scales, F^R = -F0^R sum_k u^(k) e^{i k.x} over the
// damped shell, recomputed every step from the bare velocity j/rho.
//
// One damped step is two launches (the coefficient stage below runs inside
// the step kernel; the moment kernel has it as a launch of its own):
//  1. k_edm_fourier: each workgroup pulls the pre-collision populations of a
//     block of 256 columns and `rows` rows, forms u = j/rho and reduces the
//     Fourier sums C_k = sum u cos(k.x), S_k = sum u sin(k.x) of both
//     components over its sites (first along y per column against the y
//     tables, then per mode against the column's x tables, summed over the
//     workgroup) into 4 m partials.
//  2. coefficients: the partials are added in a fixed order (edm_sums) and the
//     sums turned into per-row coefficients (edm_row_coef): with
//     theta = kx phi + ky beta,
//       F^R(x, y) = sum_{m = 0..km} A_m(y) cos(m phi) + B_m(y) sin(m phi),
//     A_m = -2 F0 sum_{|kx| = m} (C cos ky beta + S sin ky beta),
//     B_m = -2 F0 sum_{|kx| = m} sgn(kx) (S cos ky beta - C sin ky beta)
//     (each mode of the half plane stands for itself and its conjugate -k).
//  3. k_edm_step: pull, moments, force F = F_ext + F^R, exact-difference
//     collision, store; same memory traffic as the Guo step.
// Without damping only the step kernel runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lbm_internal.h"
#include "lbm_reduce.h"
#include "lbm_site.h"

namespace lbm {
namespace {

using namespace step_detail;
using namespace reduce_detail;

// Fourier launch: workgroups of kFourierCols threads, one column each, over
// `rows` consecutive rows; at most 1024 workgroups.  The coefficient kernel is
// one workgroup of kCoefThreads threads.
constexpr int kFourierCols = 256;
constexpr int kCoefThreads = 1024;
constexpr int kEdmTileRows = 64;

int dft_xblocks(int nx) { return (nx + kFourierCols - 1) / kFourierCols; }
// at least 4 rows per workgroup (fewer partials to add), at most 1024 workgroups
int dft_rows(int nx, int ny) {
  const long long r = (static_cast<long long>(ny) * dft_xblocks(nx) + 1023) / 1024;
  return static_cast<int>(std::min<long long>(ny, std::max<long long>(4, r)));
}
int dft_blocks(int nx, int ny) {
  const int r = dft_rows(nx, ny);
  return dft_xblocks(nx) * ((ny + r - 1) / r);
}

// cos and sin of 2 pi m x / n for m = 0..km, from the exact integer residue.
template <typename T>
__global__ void __launch_bounds__(256) k_edm_tables(double* __restrict__ tabx, double* __restrict__ taby,
                                                    T* __restrict__ tabx_t, int nx, int ny, int km) {
  const int nxx = (km + 1) * nx, total = nxx + (km + 1) * ny;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const bool isx = i < nxx;
    const int j = isx ? i : i - nxx;
    const int n = isx ? nx : ny;
    const int m = j / n, x = j % n;
    const int r = static_cast<int>((static_cast<long long>(m) * x) % n);
    double sv, cv;
    sincospi(2.0 * r / n, &sv, &cv);
    double* tab = isx ? tabx : taby;
    tab[(2 * m) * n + x] = cv;
    tab[(2 * m + 1) * n + x] = sv;
    if (isx) {
      tabx_t[(2 * m) * n + x] = T(cv);
      tabx_t[(2 * m + 1) * n + x] = T(sv);
    }
  }
}

// rho, j and 1/rho of one site from the deviations d_l = f_l - w_l (the sums
// are grouped as in the Guo step).
template <typename T>
struct EdmSite {
  T drho, rho, jx, jy, inv;
  __device__ __forceinline__ explicit EdmSite(const T (&d)[9]) {
    drho = ((d[0] + (d[1] + d[3])) + (d[2] + d[4])) + ((d[5] + d[7]) + (d[6] + d[8]));
    rho = T(1) + drho;
    jx = (d[1] - d[3]) + ((d[5] - d[7]) + (d[8] - d[6]));
    jy = (d[2] - d[4]) + ((d[5] - d[7]) + (d[6] - d[8]));
    inv = recip<T>(rho);
  }
};

// F^R at one site from the row's coefficients cr[(m, {Ax, Bx, Ay, By})] and the
// column's cos(m phi), sin(m phi).
template <typename T, int KM>
__device__ __forceinline__ void damp_force(const T* __restrict__ cr, const T (&cm)[KM + 1],
                                           const T (&sm)[KM + 1], T& fx, T& fy) {
  T ax = cr[0], ay = cr[2];
#pragma unroll
  for (int m = 1; m <= KM; ++m) {
    ax += cr[4 * m] * cm[m] + cr[4 * m + 1] * sm[m];
    ay += cr[4 * m + 2] * cm[m] + cr[4 * m + 3] * sm[m];
  }
  fx += ax;
  fy += ay;
}

// Exact-difference collision in deviation form: with u = j/rho and
// v = u + F/rho, f* = (1 - omega)(f - f^eq(u)) + f^eq(v), i.e.
//   f*_l = (1 - omega) d_l + S + A,  f*_lbar = (1 - omega) d_lbar + S - A,
//   S = w (B + 4.5 rho ((c.v)^2 - (1 - omega)(c.u)^2)),
//   A = 3 w rho (c.v - (1 - omega) c.u),
//   B = omega drho - 1.5 rho (|v|^2 - (1 - omega)|u|^2).
template <typename T>
__device__ __forceinline__ void edm_collide(const T (&d)[9], const EdmSite<T>& s, T ux, T uy, T vx,
                                            T vy, T omega, T (&o)[9]) {
  const T om1 = T(1) - omega;
  const T B = omega * s.drho - T(1.5) * s.rho * ((vx * vx + vy * vy) - om1 * (ux * ux + uy * uy));
  const T r45 = T(4.5) * s.rho, r3 = T(3) * s.rho;
  o[0] = om1 * d[0] + T(wq(0)) * B;
  auto pair = [&](int l, int lb, T cu, T cv, T w) {
    const T S = w * (B + r45 * (cv * cv - om1 * (cu * cu)));
    const T A = (w * r3) * (cv - om1 * cu);
    o[l] = om1 * d[l] + (S + A);
    o[lb] = om1 * d[lb] + (S - A);
  };
  const T wa = T(wq(1)), wd = T(wq(5));
  pair(1, 3, ux, vx, wa);
  pair(2, 4, uy, vy, wa);
  pair(5, 7, ux + uy, vx + vy, wd);
  pair(6, 8, uy - ux, vy - vx, wd);
}

// ---- 1. Fourier sums of the bare velocity ----------------------------------------
// Per thread (one column x, rows y0..y1): Uc[n] = sum_y u cos(n beta_y) and
// Us[n] = sum_y u sin(n beta_y) for n = 0..KM and both components; then per
// mode k = (kx, ky), with alpha = kx phi_x,
//   C_k += cos(alpha) Uc[ky] - sin(alpha) Us[ky],  S_k += sin(alpha) Uc[ky] + cos(alpha) Us[ky],
// reduced over the wavefront by shuffles and over the workgroup's wavefronts
// in LDS, both in a fixed order.
template <typename T, int KM>
__global__ void __launch_bounds__(kFourierCols) k_edm_fourier(const T* __restrict__ pop, size_t ps, size_t rs,
                                                              int nx, int ny, int rows, int xblocks,
                                                              const double* __restrict__ tabx,
                                                              const double* __restrict__ taby, EdmModes md,
                                                              double* __restrict__ partials, size_t pop_stride) {
  constexpr int K1 = KM + 1;
  constexpr int kWaves = kFourierCols / 64;
  pop += blockIdx.y * pop_stride;  // run blockIdx.y
  partials += static_cast<size_t>(blockIdx.y) * gridDim.x * 4 * md.m;
  __shared__ double wsum[kWaves][4 * kEdmMaxModes];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int xb = blockIdx.x % xblocks, yc = blockIdx.x / xblocks;
  const int x = xb * kFourierCols + tid;
  const int y0 = yc * rows, y1 = min(ny, y0 + rows);
  double ucx[K1], usx[K1], ucy[K1], usy[K1];
#pragma unroll
  for (int n = 0; n < K1; ++n) ucx[n] = usx[n] = ucy[n] = usy[n] = 0.0;
  double cx[K1], sx[K1];
  cx[0] = 1.0;
  sx[0] = 0.0;
#pragma unroll
  for (int m = 1; m < K1; ++m) {
    cx[m] = x < nx ? tabx[(2 * m) * nx + x] : 0.0;
    sx[m] = x < nx ? tabx[(2 * m + 1) * nx + x] : 0.0;
  }
  if (x < nx) {
    // rows in groups of four, the group's loads issued together; the sums still
    // run row by row
    for (int yg = y0; yg < y1; yg += 4) {
      T d[4][9][1];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int y = min(yg + q, y1 - 1);
        const int yn = (y == 0) ? ny - 1 : y - 1;
        const int yp = (y == ny - 1) ? 0 : y + 1;
        pull_all<T, 1>(pop, ps, rs, nx, x, y, yn, yp, d[q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int y = yg + q;
        if (y >= y1) break;
        T di[9];
#pragma unroll
        for (int l = 0; l < 9; ++l) di[l] = d[q][l][0];
        const EdmSite<T> st(di);
        const double ux = double(st.jx * st.inv), uy = double(st.jy * st.inv);
#pragma unroll
        for (int n = 0; n < K1; ++n) {
          const double c = taby[(2 * n) * ny + y], sn = taby[(2 * n + 1) * ny + y];
          ucx[n] += ux * c;
          usx[n] += ux * sn;
          ucy[n] += uy * c;
          usy[n] += uy * sn;
        }
      }
    }
  }
  // modes in groups of four: the 16 wavefront reductions of a group are independent
  // chains of shuffles that the compiler interleaves
  for (int k0 = 0; k0 < md.m; k0 += 4) {
    double v[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + j < md.m ? k0 + j : k0;
      const int kx = md.kx[k], ky = md.ky[k];
      const int mk = kx < 0 ? -kx : kx;
      double ca = 0.0, sa = 0.0, a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
      for (int n = 0; n < K1; ++n) {
        ca = n == mk ? cx[n] : ca;
        sa = n == mk ? sx[n] : sa;
        a0 = n == ky ? ucx[n] : a0;
        a1 = n == ky ? usx[n] : a1;
        b0 = n == ky ? ucy[n] : b0;
        b1 = n == ky ? usy[n] : b1;
      }
      if (kx < 0) sa = -sa;
      v[j][0] = ca * a0 - sa * a1;
      v[j][1] = sa * a0 + ca * a1;
      v[j][2] = ca * b0 - sa * b1;
      v[j][3] = sa * b0 + ca * b1;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[j][q] = wave_sum(v[j][q]);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k0 + j < md.m)
#pragma unroll
          for (int q = 0; q < 4; ++q) wsum[wave][4 * (k0 + j) + q] = v[j][q];
    }
  }
  __syncthreads();
  const int V = 4 * md.m;
  if (tid < V) {
    double a = wsum[0][tid];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) a += wsum[w][tid];
    partials[static_cast<size_t>(blockIdx.x) * V + tid] = a;
  }
}

// ---- 2. coefficients ---------------------------------------------------------------------
// cf[v] = sum over the nparts partials of value v, in an order that does not
// depend on the workgroup's size: eight interleaved running sums
// (b = j, j + 8, ...) added as ((0 + 1) + (2 + 3)) + ((4 + 5) + (6 + 7)).
// part is LDS scratch of 8 x V doubles; every thread of the workgroup calls it.
__device__ __forceinline__ void edm_sums(const double* __restrict__ partials, int nparts, int V,
                                         double* part, double* cf) {
  const int nt = blockDim.x * blockDim.y;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  for (int q = tid; q < 8 * V; q += nt) {
    const int v = q % V, j = q / V;
    double a = 0.0;
    int b = j;
    for (; b + 56 < nparts; b += 64) {  // eight loads in flight, added in order
      double t[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) t[i] = partials[static_cast<size_t>(b + 8 * i) * V + v];
#pragma unroll
      for (int i = 0; i < 8; ++i) a += t[i];
    }
    for (; b < nparts; b += 8) a += partials[static_cast<size_t>(b) * V + v];
    part[j * V + v] = a;
  }
  __syncthreads();
  for (int v = tid; v < V; v += nt) {
    const double* p = part + v;
    cf[v] = ((p[0] + p[V]) + (p[2 * V] + p[3 * V])) + ((p[4 * V] + p[5 * V]) + (p[6 * V] + p[7 * V]));
  }
  __syncthreads();
}

// The coefficients (A_x, B_x, A_y, B_y) per m = 0..KM of row y, from the sums cf.
template <typename T, int KM>
__device__ __forceinline__ void edm_row_coef(const double* cf, const double* __restrict__ taby,
                                             const EdmModes& md, int ny, int y, double scale, T* out) {
  constexpr int K1 = KM + 1;
  double cb[K1], sb[K1];
#pragma unroll
  for (int n = 0; n < K1; ++n) {
    cb[n] = taby[(2 * n) * ny + y];
    sb[n] = taby[(2 * n + 1) * ny + y];
  }
  double A[2][K1], B[2][K1];
#pragma unroll
  for (int m = 0; m < K1; ++m) A[0][m] = A[1][m] = B[0][m] = B[1][m] = 0.0;
  for (int k = 0; k < md.m; ++k) {
    const int kx = md.kx[k], ky = md.ky[k];
    const int mk = kx < 0 ? -kx : kx;
    const double sg = kx < 0 ? -1.0 : (kx > 0 ? 1.0 : 0.0);
    double c = 0.0, sn = 0.0;
#pragma unroll
    for (int n = 0; n < K1; ++n) {
      c = n == ky ? cb[n] : c;
      sn = n == ky ? sb[n] : sn;
    }
#pragma unroll
    for (int m = 0; m < K1; ++m) {
      if (m != mk) continue;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double C = cf[4 * k + 2 * q], S = cf[4 * k + 2 * q + 1];
        A[q][m] += C * c + S * sn;
        B[q][m] += sg * (S * c - C * sn);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < K1; ++m) {
    out[4 * m] = T(scale * A[0][m]);
    out[4 * m + 1] = T(scale * B[0][m]);
    out[4 * m + 2] = T(scale * A[1][m]);
    out[4 * m + 3] = T(scale * B[1][m]);
  }
}

// Per-run damping rates of a launch.
struct EdmRates {
  double f0[kEdmMaxRuns];
};

// One workgroup per run (blockIdx.x): every row's coefficients into coef (the
// moment kernel's input).
template <typename T, int KM>
__global__ void __launch_bounds__(kCoefThreads) k_edm_coef(const double* __restrict__ partials, int nparts,
                                                              const double* __restrict__ taby, EdmModes md,
                                                              int ny, T* __restrict__ coef, EdmRates rates) {
  constexpr int K1 = KM + 1;
  __shared__ double part[8 * 4 * kEdmMaxModes];
  __shared__ double cf[4 * kEdmMaxModes];
  const int V = 4 * md.m;
  partials += static_cast<size_t>(blockIdx.x) * nparts * V;
  coef += static_cast<size_t>(blockIdx.x) * ny * K1 * 4;
  edm_sums(partials, nparts, V, part, cf);
  const double scale = -2.0 * rates.f0[blockIdx.x];
  for (int y = threadIdx.x; y < ny; y += kCoefThreads)
    edm_row_coef<T, KM>(cf, taby, md, ny, y, scale, coef + static_cast<size_t>(y) * K1 * 4);
}

// ---- 3. the step ---------------------------------------------------------------------
// Same tiling as the Guo single step with one site per thread: a workgroup
// of blockDim.x x blockDim.y threads covers blockDim.x columns and
// blockDim.y * ry rows; consecutive tiles on one XCD.
// Per-run values of a step launch (run = blockIdx.y).
struct EdmStepRuns {
  size_t pop_stride, force_stride;
  double omega[kEdmMaxRuns];
  double f0[kEdmMaxRuns];
};
// With damping on a small grid (partials given), each workgroup first adds
// the run's Fourier partials itself (edm_sums, the coefficient kernel's
// order) and forms the coefficients of its tile's rows in LDS (at most
// kEdmTileRows rows); otherwise it reads them from coef, which the
// coefficient kernel wrote.
template <typename T, int KM, bool FT, bool DAMP, bool NT>
__global__ void __launch_bounds__(1024) k_edm_step(StepParams p, const T* __restrict__ tabx_t,
                                                   const double* __restrict__ partials, int nparts,
                                                   const double* __restrict__ taby, const T* __restrict__ coef,
                                                   EdmModes md, int tiles_x, int total, int per_xcd, int ry,
                                                   EdmStepRuns runs) {
  const int b = blockIdx.x;
  const int tile = (b & 7) * per_xcd + (b >> 3);
  if (tile >= total) return;  // uniform over the workgroup
  const int r = blockIdx.y;
  p.src = static_cast<const T*>(p.src) + r * runs.pop_stride;
  p.dst = static_cast<T*>(p.dst) + r * runs.pop_stride;
  if constexpr (FT) {
    p.fx = static_cast<const T*>(p.fx) + r * runs.force_stride;
    p.fy = static_cast<const T*>(p.fy) + r * runs.force_stride;
  }
  p.omega = runs.omega[r];
  const int tx = tile % tiles_x;
  const int ty = tile / tiles_x;
  __shared__ T crow[DAMP ? kEdmTileRows : 1][4 * (KM + 1)];
  if constexpr (DAMP) {
    coef += static_cast<size_t>(r) * p.ny * (KM + 1) * 4;
    if (partials) {  // uniform over the launch
      __shared__ double part[8 * 4 * kEdmMaxModes];
      __shared__ double cf[4 * kEdmMaxModes];
      const int V = 4 * md.m;
      edm_sums(partials + static_cast<size_t>(r) * nparts * V, nparts, V, part, cf);
      const int rows = blockDim.y * ry, y0 = ty * rows;
      const int tid = threadIdx.y * blockDim.x + threadIdx.x;
      for (int q = tid; q < rows; q += blockDim.x * blockDim.y)
        if (y0 + q < p.ny) edm_row_coef<T, KM>(cf, taby, md, p.ny, y0 + q, -2.0 * runs.f0[r], crow[q]);
      __syncthreads();
    }
  }
  const int x = tx * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const int ybase = (ty * blockDim.y + threadIdx.y) * ry;
  const int nx = p.nx, ny = p.ny;
  const T* __restrict__ src = static_cast<const T*>(p.src);
  T* __restrict__ dst = static_cast<T*>(p.dst);
  const T omega = T(p.omega);
  T cm[KM + 1], sm[KM + 1];
  if constexpr (DAMP) {
#pragma unroll
    for (int m = 1; m <= KM; ++m) {
      cm[m] = tabx_t[(2 * m) * nx + x];
      sm[m] = tabx_t[(2 * m + 1) * nx + x];
    }
  }
  for (int k = 0; k < ry; ++k) {
    const int y = ybase + k;
    if (y >= ny) break;
    const int yn = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    T d[9][1];
    pull_all<T, 1>(src, p.ps, p.rs, nx, x, y, yn, yp, d);
    T di[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) di[l] = d[l][0];
    const size_t i = static_cast<size_t>(y) * nx + x;
    T Fx = T(0), Fy = T(0);
    if constexpr (FT) {
      Fx = static_cast<const T*>(p.fx)[i];
      Fy = static_cast<const T*>(p.fy)[i];
    }
    if constexpr (DAMP)
      damp_force<T, KM>(partials ? crow[threadIdx.y * ry + k] : coef + static_cast<size_t>(y) * (KM + 1) * 4, cm,
                        sm, Fx, Fy);
    const EdmSite<T> s(di);
    const T ux = s.jx * s.inv, uy = s.jy * s.inv;
    const T vx = (s.jx + Fx) * s.inv, vy = (s.jy + Fy) * s.inv;
    T o[9];
    edm_collide<T>(di, s, ux, uy, vx, vy, omega, o);
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      T* q = dst + l * p.ps + static_cast<size_t>(y) * p.rs + x;
      if constexpr (NT) __builtin_nontemporal_store(o[l], q);
      else *q = o[l];
    }
    if (p.h_rho) {
      p.h_rho[i] = 1.0 + double(s.drho);  // rho - 1 kept to the storage type's precision
      p.h_ux[i] = double((s.jx + T(0.5) * Fx) * s.inv);
      p.h_uy[i] = double((s.jy + T(0.5) * Fy) * s.inv);
    }
  }
}

// ---- moments ---------------------------------------------------------------------------
template <typename T, typename O, int KM, bool FT, bool DAMP>
__global__ void __launch_bounds__(kRedThreads) k_edm_moments(MomentParams p, const T* __restrict__ tabx_t,
                                                             const T* __restrict__ coef) {
  const int nx = p.nx, ny = p.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const T* __restrict__ pop = static_cast<const T*>(p.pop);
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 1.0e300, 0.0};
  for (size_t i = blockIdx.x * size_t(kRedThreads) + threadIdx.x; i < plane;
       i += size_t(gridDim.x) * kRedThreads) {
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
    T Fx = T(0), Fy = T(0);
    if constexpr (FT) {
      Fx = static_cast<const T*>(p.fx)[i];
      Fy = static_cast<const T*>(p.fy)[i];
    }
    if constexpr (DAMP) {
      T cm[KM + 1], sm[KM + 1];
#pragma unroll
      for (int m = 1; m <= KM; ++m) {
        cm[m] = tabx_t[(2 * m) * nx + x];
        sm[m] = tabx_t[(2 * m + 1) * nx + x];
      }
      damp_force<T, KM>(coef + static_cast<size_t>(y) * (KM + 1) * 4, cm, sm, Fx, Fy);
    }
    const EdmSite<T> s(d);
    const T ux = (s.jx + T(0.5) * Fx) * s.inv, uy = (s.jy + T(0.5) * Fy) * s.inv;
    const double r = 1.0 + double(s.drho), vx = ux, vy = uy;  // rho formed in FP64
    if (p.rho) static_cast<O*>(p.rho)[i] = O(r);
    if (p.ux) static_cast<O*>(p.ux)[i] = O(ux);
    if (p.uy) static_cast<O*>(p.uy)[i] = O(uy);
    if (p.rho64) {
      p.rho64[i] = r;
      p.ux64[i] = vx;
      p.uy64[i] = vy;
    }
    if (p.ftx64) {
      p.ftx64[i] = double(Fx);
      p.fty64[i] = double(Fy);
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

// ---- host side ---------------------------------------------------------------------------
size_t esize(int dtype) { return dtype == LBM_F64 ? 8 : 4; }

// The Fourier sums of runs.n runs (run 0's populations at pop) into w.partials.
template <typename T, int KM>
int launch_sums(const lbm_config& c, const EdmWs& w, const EdmModes& md, const EdmRuns& runs,
                const void* pop, size_t ps, size_t rs, hipStream_t s) {
  const int nb = dft_blocks(c.nx, c.ny);
  hipLaunchKernelGGL((k_edm_fourier<T, KM>), dim3(nb, runs.n), dim3(kFourierCols), 0, s,
                     static_cast<const T*>(pop), ps, rs, c.nx, c.ny, dft_rows(c.nx, c.ny), dft_xblocks(c.nx),
                     w.tabx, w.taby, md, w.partials, runs.pop_stride);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

// The Fourier sums and every row's coefficients of runs.n runs.
template <typename T, int KM>
int launch_fourier(const lbm_config& c, const EdmWs& w, const EdmModes& md, const EdmRuns& runs,
                   const void* pop, size_t ps, size_t rs, hipStream_t s) {
  if (int rc = launch_sums<T, KM>(c, w, md, runs, pop, ps, rs, s)) return rc;
  const int nb = dft_blocks(c.nx, c.ny);
  EdmRates rates{};
  for (int r = 0; r < runs.n; ++r) rates.f0[r] = runs.f0[r];
  hipLaunchKernelGGL((k_edm_coef<T, KM>), dim3(runs.n), dim3(kCoefThreads), 0, s, w.partials, nb, w.taby, md,
                     c.ny, static_cast<T*>(w.coef), rates);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

// One run: its own 1/tau and damping rate, no strides.
EdmRuns single_run(const EdmModes& md, double omega) {
  EdmRuns r;
  r.omega[0] = omega;
  r.f0[0] = md.f0;
  return r;
}

template <typename T, int KM, bool FT, bool DAMP>
int launch_step_k(const lbm_config& c, const EdmWs& w, const EdmModes& md, const EdmRuns& runs,
                  const StepParams& p, const lbm_tile& t, hipStream_t s) {
  const int tiles_x = (p.nx + t.bx - 1) / t.bx;
  const int rows_per_tile = t.by * t.ry;
  const int tiles_y = (p.ny + rows_per_tile - 1) / rows_per_tile;
  const int total = tiles_x * tiles_y;
  // the step's workgroups add the partials themselves while all of them read
  // at most 8 MiB per run; else one coefficient launch first
  const int nb = DAMP ? dft_blocks(c.nx, c.ny) : 0;
  const bool in_step = DAMP && static_cast<double>(nb) * total * 4 * md.m * 8 <= 8.0 * (1 << 20);
  if constexpr (DAMP) {
    if (in_step) {
      if (int rc = launch_sums<T, KM>(c, w, md, runs, p.src, p.ps, p.rs, s)) return rc;
    } else if (int rc = launch_fourier<T, KM>(c, w, md, runs, p.src, p.ps, p.rs, s)) {
      return rc;
    }
  }
  const int per_xcd = (total + 7) / 8;
  const T* tabx_t = static_cast<const T*>(w.tabx_t);
  EdmStepRuns sr{};
  sr.pop_stride = runs.pop_stride;
  sr.force_stride = runs.force_stride;
  for (int r = 0; r < runs.n; ++r) {
    sr.omega[r] = runs.omega[r];
    sr.f0[r] = runs.f0[r];
  }
  const dim3 grid(per_xcd * 8, runs.n);
  const double* parts = in_step ? w.partials : nullptr;
  const T* coef = static_cast<const T*>(w.coef);
  if (t.nt)
    hipLaunchKernelGGL((k_edm_step<T, KM, FT, DAMP, true>), grid, dim3(t.bx, t.by), 0, s, p, tabx_t, parts,
                       nb, w.taby, coef, md, tiles_x, total, per_xcd, t.ry, sr);
  else
    hipLaunchKernelGGL((k_edm_step<T, KM, FT, DAMP, false>), grid, dim3(t.bx, t.by), 0, s, p, tabx_t, parts,
                       nb, w.taby, coef, md, tiles_x, total, per_xcd, t.ry, sr);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

template <typename T, int KM, bool FT, bool DAMP>
int launch_moments_k(const lbm_config& c, const EdmWs& w, const EdmModes& md, const MomentParams& p,
                     hipStream_t s) {
  if constexpr (DAMP)
    if (int rc = launch_fourier<T, KM>(c, w, md, single_run(md, 0.0), p.pop, p.ps, p.rs, s)) return rc;
  const int g = moment_blocks(p.nx, p.ny);
  const T* tabx_t = static_cast<const T*>(w.tabx_t);
  const T* coef = static_cast<const T*>(w.coef);
  if (p.out_dtype == LBM_F32)
    hipLaunchKernelGGL((k_edm_moments<T, float, KM, FT, DAMP>), dim3(g), dim3(kRedThreads), 0, s, p, tabx_t,
                       coef);
  else
    hipLaunchKernelGGL((k_edm_moments<T, double, KM, FT, DAMP>), dim3(g), dim3(kRedThreads), 0, s, p, tabx_t,
                       coef);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

struct StepGo {
  const lbm_config& c;
  const EdmWs& w;
  const EdmModes& md;
  const EdmRuns& runs;
  const StepParams& p;
  const lbm_tile& t;
  hipStream_t s;
  template <typename T, int KM, bool FT, bool DAMP>
  int run() const {
    return launch_step_k<T, KM, FT, DAMP>(c, w, md, runs, p, t, s);
  }
};

struct MomGo {
  const lbm_config& c;
  const EdmWs& w;
  const EdmModes& md;
  const MomentParams& p;
  hipStream_t s;
  template <typename T, int KM, bool FT, bool DAMP>
  int run() const {
    return launch_moments_k<T, KM, FT, DAMP>(c, w, md, p, s);
  }
};

// Calls f.run<T, KM, FT, DAMP>() for the handle's variant.
template <typename F>
int dispatch(const lbm_config& c, const EdmModes& md, const F& f) {
  const bool ft = c.has_force != 0;
  auto by_t = [&](auto tag) -> int {
    using T = decltype(tag);
    if (md.m == 0) return ft ? f.template run<T, 0, true, false>() : f.template run<T, 0, false, false>();
    switch (md.km) {
      case 1: return ft ? f.template run<T, 1, true, true>() : f.template run<T, 1, false, true>();
      case 2: return ft ? f.template run<T, 2, true, true>() : f.template run<T, 2, false, true>();
      case 3: return ft ? f.template run<T, 3, true, true>() : f.template run<T, 3, false, true>();
      case 4: return ft ? f.template run<T, 4, true, true>() : f.template run<T, 4, false, true>();
      default: return fail(LBM_E_INVALID, "damped shell reaches |k| = %d > %d", md.km, kEdmMaxK);
    }
  };
  return c.dtype == LBM_F64 ? by_t(double{}) : by_t(float{});
}

}  // namespace

int edm_modes(const lbm_config& c, EdmModes* out) {
  EdmModes md;
  if (c.force_scheme == LBM_FORCE_EDM && c.damp_f0 > 0.0) {
    // per unnormalised Fourier sum: F^R = -(damp_f0 / (nx ny)) sum_k (sum_x u e^{-ik.x}) e^{ik.x}
    md.f0 = c.damp_f0 / (static_cast<double>(c.nx) * c.ny);
    const double lo = c.damp_kmin * c.damp_kmin, hi = c.damp_kmax * c.damp_kmax;
    for (int ky = 0; ky <= kEdmMaxK; ++ky)
      for (int kx = -kEdmMaxK; kx <= kEdmMaxK; ++kx) {
        if (ky == 0 && kx <= 0) continue;
        const double k2 = double(kx * kx + ky * ky);
        if (k2 < lo || k2 > hi) continue;
        if (md.m == kEdmMaxModes) return fail(LBM_E_INVALID, "more than %d damped modes", kEdmMaxModes);
        md.kx[md.m] = static_cast<int8_t>(kx);
        md.ky[md.m] = static_cast<int8_t>(ky);
        md.km = std::max(md.km, std::max(kx < 0 ? -kx : kx, ky));
        ++md.m;
      }
    if (md.m == 0)
      return fail(LBM_E_INVALID, "no integer wavevector with %g <= |k| <= %g", c.damp_kmin, c.damp_kmax);
  }
  *out = md;
  return LBM_OK;
}

EdmWs carve_edm(Carver& cv, const lbm_config& c, const EdmModes& md) { return carve_edm_runs(cv, c, md, 1); }

EdmWs carve_edm_runs(Carver& cv, const lbm_config& c, const EdmModes& md, int nruns) {
  EdmWs w;
  if (c.force_scheme != LBM_FORCE_EDM || md.m == 0) return w;
  const size_t k1 = static_cast<size_t>(md.km) + 1, es = esize(c.dtype);
  w.tabx = cv.take<double>(k1 * 2 * c.nx);
  w.taby = cv.take<double>(k1 * 2 * c.ny);
  w.tabx_t = cv.take<char>(k1 * 2 * c.nx * es);
  w.partials = cv.take<double>(static_cast<size_t>(nruns) * dft_blocks(c.nx, c.ny) * 4 * md.m);
  w.coef = cv.take<char>(static_cast<size_t>(nruns) * c.ny * k1 * 4 * es);
  return w;
}

EdmWs edm_run_view(const EdmWs& w, const lbm_config& c, const EdmModes& md, int r) {
  EdmWs v = w;
  if (md.m == 0) return v;
  const size_t k1 = static_cast<size_t>(md.km) + 1;
  v.partials = w.partials + static_cast<size_t>(r) * dft_blocks(c.nx, c.ny) * 4 * md.m;
  v.coef = static_cast<char*>(w.coef) + static_cast<size_t>(r) * c.ny * k1 * 4 * esize(c.dtype);
  return v;
}

int edm_tables(const lbm_config& c, const EdmWs& w, const EdmModes& md, hipStream_t s) {
  if (md.m == 0) return LBM_OK;
  const int n = (md.km + 1) * (c.nx + c.ny);
  const int g = std::min(1024, (n + 255) / 256);
  if (c.dtype == LBM_F64)
    hipLaunchKernelGGL(k_edm_tables<double>, dim3(g), dim3(256), 0, s, w.tabx, w.taby,
                       static_cast<double*>(w.tabx_t), c.nx, c.ny, md.km);
  else
    hipLaunchKernelGGL(k_edm_tables<float>, dim3(g), dim3(256), 0, s, w.tabx, w.taby,
                       static_cast<float*>(w.tabx_t), c.nx, c.ny, md.km);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

bool edm_tile_ok(const lbm_tile& t, int nx, int ny) {
  (void)nx;
  (void)ny;
  if (t.fuse < 0 || t.fuse > 1 || t.vx != 1 || t.pf != 0 || t.halo != 0) return false;
  const int threads = t.bx * t.by;
  if (t.bx < 1 || t.by < 1 || t.ry < 1 || threads > 1024 || threads % 64 != 0) return false;
  if (t.by * t.ry > kEdmTileRows) return false;  // the step kernel's rows of coefficients in LDS
  return t.nt == 0 || t.nt == 1;
}

lbm_tile edm_default_tile(int nx) {
  lbm_tile t{};
  int bx = 64;
  while (bx < 256 && bx * 2 <= nx) bx *= 2;
  t.bx = bx;
  t.by = 256 / bx;
  t.vx = 1;
  t.ry = 1;
  t.nt = 0;
  t.fuse = 1;
  t.pf = 0;
  return t;
}

int edm_step(const lbm_config& c, const EdmWs& w, const EdmModes& md, const StepParams& p,
             const lbm_tile& t, hipStream_t s) {
  if (!edm_tile_ok(t, c.nx, c.ny))
    return fail(LBM_E_INVALID, "invalid launch shape for the exact-difference step");
  const EdmRuns one = single_run(md, p.omega);
  return dispatch(c, md, StepGo{c, w, md, one, p, t, s});
}

int edm_step_runs(const lbm_config& c, const EdmWs& w, const EdmModes& md, const EdmRuns& runs,
                  const StepParams& p, const lbm_tile& t, hipStream_t s) {
  if (!edm_tile_ok(t, c.nx, c.ny))
    return fail(LBM_E_INVALID, "invalid launch shape for the exact-difference step");
  if (runs.n < 1 || runs.n > kEdmMaxRuns) return fail(LBM_E_INVALID, "1..%d runs per launch", kEdmMaxRuns);
  if (p.h_rho) return fail(LBM_E_INVALID, "no moment record in a batched step");
  return dispatch(c, md, StepGo{c, w, md, runs, p, t, s});
}

int edm_moments(const lbm_config& c, const EdmWs& w, const EdmModes& md, const MomentParams& p,
                hipStream_t s) {
  return dispatch(c, md, MomGo{c, w, md, p, s});
}

}  // namespace lbm
