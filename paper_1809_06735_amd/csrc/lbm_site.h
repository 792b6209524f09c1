// Per-site device arithmetic of the D2Q9 step, shared by the single-grid and
// batched kernels: vector loads with periodic pulls, moments, BGK collision
// with Guo forcing (all in deviation form f_l - w_l).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {
namespace step_detail {

// ---- vector types ---------------------------------------------------------------
template <typename T, int VX> struct Vec;
template <> struct Vec<float, 2> {
  typedef float A __attribute__((ext_vector_type(2), aligned(8)));
  typedef float U __attribute__((ext_vector_type(2), aligned(4)));
};
template <> struct Vec<float, 4> {
  typedef float A __attribute__((ext_vector_type(4), aligned(16)));
  typedef float U __attribute__((ext_vector_type(4), aligned(4)));
};
template <> struct Vec<double, 2> {
  typedef double A __attribute__((ext_vector_type(2), aligned(16)));
  typedef double U __attribute__((ext_vector_type(2), aligned(8)));
};
template <> struct Vec<double, 4> {
  typedef double A __attribute__((ext_vector_type(4), aligned(32)));
  typedef double U __attribute__((ext_vector_type(4), aligned(8)));
};

// o[i] = row[(x0 + i - cx) mod nx], i < VX; x0 is a multiple of VX.
template <typename T, int VX, int CX>
__device__ __forceinline__ void pull_row(const T* __restrict__ row, int x0, int nx, T (&o)[VX]) {
  if constexpr (VX == 1) {
    int xs = x0 - CX;
    if (CX == 1 && xs < 0) xs += nx;
    if (CX == -1 && xs >= nx) xs -= nx;
    o[0] = row[xs];
  } else {
    typedef typename Vec<T, VX>::A VA;
    typedef typename Vec<T, VX>::U VU;
    if constexpr (CX == 0) {
      VA v = *reinterpret_cast<const VA*>(row + x0);
#pragma unroll
      for (int i = 0; i < VX; ++i) o[i] = v[i];
    } else if constexpr (CX == 1) {
      if (x0 > 0) {
        VU v = *reinterpret_cast<const VU*>(row + x0 - 1);
#pragma unroll
        for (int i = 0; i < VX; ++i) o[i] = v[i];
      } else {
        VA v = *reinterpret_cast<const VA*>(row);
        o[0] = row[nx - 1];
#pragma unroll
        for (int i = 1; i < VX; ++i) o[i] = v[i - 1];
      }
    } else {
      if (x0 + VX < nx) {
        VU v = *reinterpret_cast<const VU*>(row + x0 + 1);
#pragma unroll
        for (int i = 0; i < VX; ++i) o[i] = v[i];
      } else {
        VA v = *reinterpret_cast<const VA*>(row + x0);
#pragma unroll
        for (int i = 0; i < VX - 1; ++i) o[i] = v[i + 1];
        o[VX - 1] = row[0];
      }
    }
  }
}

template <typename T, int VX>
__device__ __forceinline__ void load_aligned(const T* __restrict__ p, T (&o)[VX]) {
  if constexpr (VX == 1) {
    o[0] = *p;
  } else {
    typedef typename Vec<T, VX>::A VA;
    VA v = *reinterpret_cast<const VA*>(p);
#pragma unroll
    for (int i = 0; i < VX; ++i) o[i] = v[i];
  }
}

template <typename T, int VX, bool NT>
__device__ __forceinline__ void store_aligned(T* __restrict__ p, const T (&o)[VX]) {
  if constexpr (VX == 1) {
    if constexpr (NT) __builtin_nontemporal_store(o[0], p);
    else *p = o[0];
  } else {
    typedef typename Vec<T, VX>::A VA;
    VA v;
#pragma unroll
    for (int i = 0; i < VX; ++i) v[i] = o[i];
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<VA*>(p));
    else *reinterpret_cast<VA*>(p) = v;
  }
}

// 1/x: IEEE division in FP64; in FP32 the hardware reciprocal refined by one
// Newton step (within an ulp of the quotient, a third of the instructions).
template <typename T>
__device__ __forceinline__ T recip(T x) {
  if constexpr (sizeof(T) == 4) {
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
  } else {
    return T(1) / x;
  }
}

// Pre-collision moments of one site from the deviations d_l = f_l - w_l.
// rho = 1 + sum d; j = sum c d; half-force velocity with implicit drag:
// u = (j + F_ext/2) / (rho (1 + alpha/2)), total force F = F_ext - alpha rho u.
template <typename T, bool FORCE>
struct SiteMoments {
  T drho, rho, ux, uy, Fx, Fy;
  __device__ __forceinline__ SiteMoments(const T (&d)[9], T fx, T fy, T alpha) {
    drho = ((d[0] + (d[1] + d[3])) + (d[2] + d[4])) + ((d[5] + d[7]) + (d[6] + d[8]));
    rho = T(1) + drho;
    const T jx = (d[1] - d[3]) + ((d[5] - d[7]) + (d[8] - d[6]));
    const T jy = (d[2] - d[4]) + ((d[5] - d[7]) + (d[6] - d[8]));
    if constexpr (FORCE) {
      const T inv = recip<T>(rho * (T(1) + T(0.5) * alpha));
      ux = (jx + T(0.5) * fx) * inv;
      uy = (jy + T(0.5) * fy) * inv;
      Fx = fx - alpha * rho * ux;
      Fy = fy - alpha * rho * uy;
    } else {
      const T inv = recip<T>(rho);
      ux = jx * inv;
      uy = jy * inv;
      Fx = T(0);
      Fy = T(0);
    }
  }
};

// BGK collision (Eq. 1) towards the equilibrium of Eq. 2, with Guo's forcing
// term (1 - 1/(2 tau)) w [3 (c - u) + 9 (c.u) c] . F, all in deviation form:
// f* = (1 - omega) d + omega d^eq + G.  Opposite velocities l, lbar share w
// and the parts of omega d^eq + G that are even in c, and see the odd parts
// with opposite signs.  With cu = c.u, cF = c.F, g = 1 - omega/2:
//   even  S = w B0 + 3 w cu (1.5 omega rho cu + 3 g cF),
//         B0 = omega (drho - 1.5 rho |u|^2) - 3 g u.F,
//   odd   A = w (3 omega rho cu + 3 g cF),
// and f*_l = (1 - omega) d_l + S + A, f*_lbar = (1 - omega) d_lbar + S - A.
// Without a force F = 0 and the same terms are grouped by powers of cu.
template <typename T, bool FORCE>
__device__ __forceinline__ void collide_site(const T (&d)[9], const SiteMoments<T, FORCE>& m,
                                             T omega, T guo, T (&o)[9]) {
  const T ux = m.ux, uy = m.uy;
  const T om1 = T(1) - omega;
  const T b = m.drho - m.rho * (T(1.5) * (ux * ux + uy * uy));
  const T wa = T(wq(1)), wd = T(wq(5));
  const T wRa = (T(3) * omega * wa) * m.rho, wRd = (T(3) * omega * wd) * m.rho;
  if constexpr (FORCE) {
    const T g3 = T(3) * guo;
    const T B0 = omega * b - g3 * (ux * m.Fx + uy * m.Fy);
    const T p3 = (T(1.5) * omega) * m.rho;
    const T wBa = wa * B0, wBd = wd * B0;
    o[0] = om1 * d[0] + T(wq(0)) * B0;
    auto pair = [&](int l, int lb, T cu, T cF, T w, T wB, T wR) {
      const T gc = g3 * cF;
      const T S = (T(3) * w) * (cu * (p3 * cu + gc)) + wB;
      const T A = wR * cu + w * gc;
      o[l] = om1 * d[l] + (S + A);
      o[lb] = om1 * d[lb] + (S - A);
    };
    pair(1, 3, ux, m.Fx, wa, wBa, wRa);
    pair(2, 4, uy, m.Fy, wa, wBa, wRa);
    pair(5, 7, ux + uy, m.Fx + m.Fy, wd, wBd, wRd);
    pair(6, 8, uy - ux, m.Fy - m.Fx, wd, wBd, wRd);
  } else {
    // S = w omega b + 4.5 w omega rho cu^2, A = 3 w omega rho cu
    const T wBa = (omega * wa) * b, wBd = (omega * wd) * b;
    const T wKa = (T(4.5) * omega * wa) * m.rho, wKd = (T(4.5) * omega * wd) * m.rho;
    o[0] = om1 * d[0] + (omega * T(wq(0))) * b;
    auto pair = [&](int l, int lb, T cu, T wB, T wK, T wR) {
      const T S = wK * (cu * cu) + wB;
      const T A = wR * cu;
      o[l] = om1 * d[l] + (S + A);
      o[lb] = om1 * d[lb] + (S - A);
    };
    pair(1, 3, ux, wBa, wKa, wRa);
    pair(2, 4, uy, wBa, wKa, wRa);
    pair(5, 7, ux + uy, wBd, wKd, wRd);
    pair(6, 8, uy - ux, wBd, wKd, wRd);
  }
}

template <int L, typename T, int VX>
__device__ __forceinline__ void pull_plane(const T* __restrict__ src, size_t ps, size_t rs, int nx,
                                           int x0, int y, int yn, int yp, T (&d)[9][VX]) {
  constexpr int cy = cyq(L);
  const int ys = cy == 1 ? yn : (cy == -1 ? yp : y);
  pull_row<T, VX, cxq(L)>(src + L * ps + static_cast<size_t>(ys) * rs, x0, nx, d[L]);
}

// Pull all nine planes of the VX sites (x0..x0+VX-1, y).
template <typename T, int VX>
__device__ __forceinline__ void pull_all(const T* __restrict__ src, size_t ps, size_t rs, int nx,
                                         int x0, int y, int yn, int yp, T (&d)[9][VX]) {
  pull_plane<0>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane<1>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane<2>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane<3>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane<4>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane<5>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane<6>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane<7>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane<8>(src, ps, rs, nx, x0, y, yn, yp, d);
}

// The transpose of the pull: d_l = a_l(x + c_l) for the VX sites (x0.., y).
template <int L, typename T, int VX>
__device__ __forceinline__ void pull_plane_rev(const T* __restrict__ src, size_t ps, size_t rs, int nx,
                                               int x0, int y, int yn, int yp, T (&d)[9][VX]) {
  constexpr int cy = cyq(L);
  const int ys = cy == 1 ? yp : (cy == -1 ? yn : y);
  pull_row<T, VX, -cxq(L)>(src + L * ps + static_cast<size_t>(ys) * rs, x0, nx, d[L]);
}

template <typename T, int VX>
__device__ __forceinline__ void pull_all_rev(const T* __restrict__ src, size_t ps, size_t rs, int nx,
                                             int x0, int y, int yn, int yp, T (&d)[9][VX]) {
  pull_plane_rev<0>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane_rev<1>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane_rev<2>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane_rev<3>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane_rev<4>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane_rev<5>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane_rev<6>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane_rev<7>(src, ps, rs, nx, x0, y, yn, yp, d);
  pull_plane_rev<8>(src, ps, rs, nx, x0, y, yn, yp, d);
}

}  // namespace step_detail
}  // namespace lbm
