// Discrete adjoint of an unforced D2Q9 BGK run with respect to the initial
// velocity field and tau, for the loss
//   J = mean over all L x L windows V of (RHS^Omega_V - LHS^Omega_V)^2
// (the enstrophy balance of Eq. 11 at the last step; a window of side
// L == nx == ny is the single whole-domain window).
//
// State convention (as in the forward step): the stored populations g^t are
// un-streamed, f^t_l(x) = g^t_l(x - c_l), and one step is g^{t+1}(x) = C(f^t(x)).
// The adjoint is kept at the site as a^t(x) = dJ/df^t(x); one backward step is
//   a^t(x) = C'(f^t(x))^T v(x) + M'(f^t(x))^T mhat^t(x),  v_l(x) = a^{t+1}_l(x + c_l),
// i.e. a pull from x + c_l (the transpose of the forward pull), where M maps
// f to (rho, u) and mhat^t are the loss seeds at t = T, T-1, T-2.  The tau
// derivative collects v . dC/dtau = v . (f - f^eq)/tau^2 per step plus the
// explicit dependence of the viscous stress on nu = (tau - 1/2)/3; the initial
// velocity gradient is (df^eq/du)^T a^0.
//
// Memory: populations are checkpointed every K steps; each segment is
// recomputed forward into a buffer of K+1 states and swept backward.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lbm_fd8.h"
#include "lbm_internal.h"
#include "lbm_site.h"

namespace lbm {
namespace {

using namespace fd8;
using namespace step_detail;

constexpr int kAT = 256;

// ---- loss: residual field and its adjoint (FP64) ---------------------------------
__global__ void __launch_bounds__(256) k_residual(const double* __restrict__ terms, size_t plane,
                                                  double* __restrict__ r) {
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < plane; i += size_t(gridDim.x) * 256)
    r[i] = (((terms[LBM_T_Z1 * plane + i] + terms[LBM_T_Z2 * plane + i]) +
             terms[LBM_T_Z3 * plane + i]) +
            (terms[LBM_T_Z4 * plane + i] + terms[LBM_T_Z5 * plane + i])) -
           terms[LBM_T_LHS_Z * plane + i];
}

__global__ void __launch_bounds__(256) k_set(double* __restrict__ out, size_t n, double v) {
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
    out[i] = v;
}

__global__ void __launch_bounds__(256) k_fill(double* __restrict__ out, size_t n, const double* v,
                                              double scale) {
  const double val = scale * v[0];
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
    out[i] = val;
}

// sum of squares of a field, block partials, then one block (deterministic)
__global__ void __launch_bounds__(256) k_sumsq(const double* __restrict__ g, size_t n,
                                               double* partials) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
    acc += g[i] * g[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ g, size_t n,
                                            double* partials) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
    acc += g[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ p, int n,
                                                      double scale, double* out) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += p[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = scale * ((sh[0] + sh[1]) + (sh[2] + sh[3]));
}

struct AdjLoss {
  const double* rho;   // level n
  const double* ux;
  const double* uy;
  const double* ux1;   // level n-1
  const double* uy1;
  const double* ux2;   // level n-2
  const double* uy2;
  const double* aux;   // balance aux fields (omega, Omega, H, sigma ...)
  const double* rhat;  // dJ/dr
  double* w;           // scratch fields [kAdjFields][plane]
  double nu;
  int nx, ny;
};

// scratch field indices
enum {
  S_W1 = 0, S_WX, S_WY, S_HTX, S_HTY, S_RHOH, S_UXD, S_UYD, S_DIV, S_OM1, S_OM2,
  S_AH, S_BH, S_CH, S_DH, S_RHON, S_NUS, S_UX1, S_UY1, S_UX2, S_UY2, S_UXN, S_UYN,
  kAdjFields
};

__device__ __forceinline__ size_t sidx(int x, int y, int nx) { return static_cast<size_t>(y) * nx + x; }

// Adjoint of the pointwise products and of the first layer of differences.
__global__ void __launch_bounds__(256) k_loss_b1(AdjLoss a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const int nx = a.nx, ny = a.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t i = sidx(x, y, nx);
  const double* W = a.aux + AUX_W * plane;
  const double rh = a.rhat[i];
  const double gx = fd8_x(F1{a.rhat, nx}, x, y, nx);
  const double gy = fd8_y(F1{a.rhat, nx}, x, y, ny);
  const double ad = fd8_x(F1{a.ux, nx}, x, y, nx);       // d_x u_x
  const double dd = fd8_y(F1{a.uy, nx}, x, y, ny);       // d_y u_y
  const double om = W[i];
  const double Om = a.aux[AUX_OM2 * plane + i];
  const double hx = a.aux[AUX_HX * plane + i];
  const double hy = a.aux[AUX_HY * plane + i];
  const double wx = fd8_x(F1{W, nx}, x, y, nx);
  const double wy = fd8_y(F1{W, nx}, x, y, ny);
  const double ux = a.ux[i], uy = a.uy[i], r = a.rho[i];
  const double div = ad + dd;
  const double Omh = gx * ux + gy * uy - rh * div - 1.5 * rh;   // dJ/dOmega (level n)
  const double hhx = gy * om + rh * wy;                          // dJ/dH_x
  const double hhy = -gx * om - rh * wx;                         // dJ/dH_y
  double* w = a.w;
  w[S_W1 * plane + i] = -gx * hy + gy * hx + Omh * om;           // dJ/domega, local part
  w[S_WX * plane + i] = -rh * hy;                                // dJ/d(d_x omega)
  w[S_WY * plane + i] = rh * hx;                                 // dJ/d(d_y omega)
  w[S_HTX * plane + i] = hhx / r;
  w[S_HTY * plane + i] = hhy / r;
  w[S_RHOH * plane + i] = -(hhx * hx + hhy * hy) / r;
  w[S_UXD * plane + i] = gx * Om;
  w[S_UYD * plane + i] = gy * Om;
  w[S_DIV * plane + i] = -rh * Om;
  const double om1 = fd8_x(F1{a.uy1, nx}, x, y, nx) - fd8_y(F1{a.ux1, nx}, x, y, ny);
  const double om2 = fd8_x(F1{a.uy2, nx}, x, y, nx) - fd8_y(F1{a.ux2, nx}, x, y, ny);
  w[S_OM1 * plane + i] = 2.0 * rh * om1;                         // dJ/domega^{n-1}
  w[S_OM2 * plane + i] = -0.5 * rh * om2;                        // dJ/domega^{n-2}
}

// Adjoint of the second layer of differences and of the viscous stress.
__global__ void __launch_bounds__(256) k_loss_b2(AdjLoss a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const int nx = a.nx, ny = a.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t i = sidx(x, y, nx);
  double* w = a.w;
  const double omh = w[S_W1 * plane + i] - fd8_x(F1{w + S_WX * plane, nx}, x, y, nx) -
                     fd8_y(F1{w + S_WY * plane, nx}, x, y, ny);
  const double* htx = w + S_HTX * plane;
  const double* hty = w + S_HTY * plane;
  const double sxx = -fd8_x(F1{htx, nx}, x, y, nx);
  const double sxy = -fd8_y(F1{htx, nx}, x, y, ny) - fd8_x(F1{hty, nx}, x, y, nx);
  const double syy = -fd8_y(F1{hty, nx}, x, y, ny);
  const double ad = fd8_x(F1{a.ux, nx}, x, y, nx);
  const double bd = fd8_y(F1{a.ux, nx}, x, y, ny);
  const double cd = fd8_x(F1{a.uy, nx}, x, y, nx);
  const double dd = fd8_y(F1{a.uy, nx}, x, y, ny);
  const double r = a.rho[i], nu = a.nu;
  const double divh = w[S_DIV * plane + i];
  w[S_AH * plane + i] = divh + 2.0 * nu * r * sxx;
  w[S_DH * plane + i] = divh + 2.0 * nu * r * syy;
  w[S_CH * plane + i] = omh + nu * r * sxy;
  w[S_BH * plane + i] = -omh + nu * r * sxy;
  w[S_RHON * plane + i] = w[S_RHOH * plane + i] + 2.0 * nu * (ad * sxx + dd * syy) + nu * (cd + bd) * sxy;
  w[S_NUS * plane + i] = r * (2.0 * ad * sxx + 2.0 * dd * syy + (cd + bd) * sxy);
  const double* o1 = w + S_OM1 * plane;
  const double* o2 = w + S_OM2 * plane;
  w[S_UX1 * plane + i] = fd8_y(F1{o1, nx}, x, y, ny);
  w[S_UY1 * plane + i] = -fd8_x(F1{o1, nx}, x, y, nx);
  w[S_UX2 * plane + i] = fd8_y(F1{o2, nx}, x, y, ny);
  w[S_UY2 * plane + i] = -fd8_x(F1{o2, nx}, x, y, nx);
}

// Adjoint of the velocity gradients at level n.
__global__ void __launch_bounds__(256) k_loss_b3(AdjLoss a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const int nx = a.nx, ny = a.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t i = sidx(x, y, nx);
  double* w = a.w;
  w[S_UXN * plane + i] = w[S_UXD * plane + i] - fd8_x(F1{w + S_AH * plane, nx}, x, y, nx) -
                         fd8_y(F1{w + S_BH * plane, nx}, x, y, ny);
  w[S_UYN * plane + i] = w[S_UYD * plane + i] - fd8_x(F1{w + S_CH * plane, nx}, x, y, nx) -
                         fd8_y(F1{w + S_DH * plane, nx}, x, y, ny);
}

// ---- population adjoint -------------------------------------------------------------
struct Seeds {
  const double* rho;  // may be null (zero)
  const double* ux;
  const double* uy;
};

template <typename T>
__device__ __forceinline__ void pull_sites(const T* __restrict__ g, PopLayout lay, int nx, int ny,
                                           int x, int y, int sign, T (&d)[9]) {
  // d_l = g_l(x - sign * c_l)
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    int xs = x - sign * cxq(l), ys = y - sign * cyq(l);
    xs += xs < 0 ? nx : 0;
    xs -= xs >= nx ? nx : 0;
    ys += ys < 0 ? ny : 0;
    ys -= ys >= ny ? ny : 0;
    d[l] = g[l * lay.ps + static_cast<size_t>(ys) * lay.rs + xs];
  }
}

// a^T(x) = M'(f^T(x))^T mhat^T(x)
template <typename T>
__global__ void __launch_bounds__(kAT) k_adj_init(const T* __restrict__ g, T* __restrict__ adj,
                                                  Seeds s, PopLayout lay, int nx, int ny) {
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t i = blockIdx.x * size_t(kAT) + threadIdx.x;
  if (i >= plane) return;
  const int x = static_cast<int>(i % nx), y = static_cast<int>(i / nx);
  T d[9];
  pull_sites<T>(g, lay, nx, ny, x, y, 1, d);
  SiteMoments<T, false> m(d, T(0), T(0), T(0));
  const double rh = s.rho ? s.rho[i] : 0.0;
  const size_t at = static_cast<size_t>(y) * lay.rs + x;
  const double ux = double(m.ux), uy = double(m.uy), rho = double(m.rho);
#pragma unroll
  for (int l = 0; l < 9; ++l)
    adj[l * lay.ps + at] = T(rh + (s.ux[i] * (cxq(l) - ux) + s.uy[i] * (cyq(l) - uy)) / rho);
}

// C'(f)^T v + M'(f)^T (rho_hat, u_hat) for one site; returns v . (f - f^eq)/tau^2.
//
// With P_l = 1 + 3 c_l.u + 4.5 (c_l.u)^2 - 1.5 |u|^2 (Eq. 2: f^eq_l = w_l rho P_l),
// the transpose of the collision's Jacobian maps v to
//   r_k = (1 - omega) v_k + omega [A + B . (c_k - u)],
//   A = sum_l w_l v_l P_l,  B = sum_l w_l v_l dP_l/du = sum_l w_l v_l (3 c_l + 9 (c_l.u) c_l - 3 u)
// (the rho of df^eq/du cancels the 1/rho of du/df).  A and B are linear in v, so
// they follow from the weighted moments of v, V = sum w v, V_a = sum w c_a v and
// V_ab = sum w c_a c_b v:  A = (1 - 1.5 |u|^2) V + 3 u.V_a + 4.5 u.V_ab.u and
// B = 3 (V_a - u V) + 9 V_ab.u.  The non-equilibrium part d_l - f^eq_l is formed
// per velocity (it is small against either term), opposite velocities sharing the
// even and odd parts of f^eq.
template <typename T, bool SEED>
__device__ __forceinline__ double adjoint_site(const T (&d)[9], const T (&v)[9], T om, double rh,
                                               double sx, double sy, T (&o)[9]) {
  SiteMoments<T, false> m(d, T(0), T(0), T(0));
  const T ux = m.ux, uy = m.uy;
  const T usq15 = T(1.5) * (ux * ux + uy * uy);
  const T wa = T(wq(1)), wd = T(wq(5));
  // weighted moments of v (axis velocities 1..4, diagonals 5..8)
  const T ax = v[1] + v[3], ay = v[2] + v[4];
  const T dp = v[5] + v[7], dm = v[6] + v[8];
  const T V0 = T(wq(0)) * v[0] + wa * (ax + ay) + wd * (dp + dm);
  const T Vx = wa * (v[1] - v[3]) + wd * ((v[5] - v[7]) + (v[8] - v[6]));
  const T Vy = wa * (v[2] - v[4]) + wd * ((v[5] - v[7]) + (v[6] - v[8]));
  const T Vxx = wa * ax + wd * (dp + dm);
  const T Vyy = wa * ay + wd * (dp + dm);
  const T Vxy = wd * (dp - dm);
  const T uVx = ux * Vxx + uy * Vxy, uVy = ux * Vxy + uy * Vyy;   // sum_l w_l v_l (c_l.u) c_l
  const T A = (T(1) - usq15) * V0 + T(3) * (ux * Vx + uy * Vy) + T(4.5) * (ux * uVx + uy * uVy);
  const T Bx = T(3) * (Vx - ux * V0) + T(9) * uVx;
  const T By = T(3) * (Vy - uy * V0) + T(9) * uVy;
  // v . (d - f^eq) in deviation form: f^eq_l - w_l = w_l (drho + rho (P_l - 1))
  const T base = m.drho - m.rho * usq15;
  const T r45 = T(4.5) * m.rho, r3 = T(3) * m.rho;
  T neq = v[0] * (d[0] - T(wq(0)) * base);
  auto pair = [&](int l, int lb, T w, T cu) {
    const T e = w * (base + r45 * cu * cu), od = w * (r3 * cu);
    neq += v[l] * ((d[l] - e) - od) + v[lb] * ((d[lb] - e) + od);
  };
  pair(1, 3, wa, ux);
  pair(2, 4, wa, uy);
  pair(5, 7, wd, ux + uy);
  pair(6, 8, wd, uy - ux);
  const T keep = T(1) - om;
  const T G = om * (A - (Bx * ux + By * uy)), Hx = om * Bx, Hy = om * By;
  const double inv_rho = SEED ? 1.0 / double(m.rho) : 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    T r = keep * v[k] + G;
    if (cxq(k) != 0) r = cxq(k) > 0 ? r + Hx : r - Hx;
    if (cyq(k) != 0) r = cyq(k) > 0 ? r + Hy : r - Hy;
    if constexpr (SEED) {
      const T ex = T(cxq(k)) - ux, ey = T(cyq(k)) - uy;
      r += T(rh + (sx * double(ex) + sy * double(ey)) * inv_rho);
    }
    o[k] = r;
  }
  return double(neq) * double(om) * double(om);
}

// Element (l, y, x) of a state in the row layout sits at (9 y + l) nx + x.  When
// a state spans less than 4 GiB, a site's byte offset fits 32 bits: each load is
// then a per-plane base (uniform, in scalar registers) plus a 32-bit lane offset
// that all nine planes share, with no 64-bit address arithmetic per access.
template <typename T>
__device__ __forceinline__ T ld_at(const T* __restrict__ plane, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_at(T* __restrict__ plane, uint32_t byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(plane) + byte_off) = v;
}

// out_l = p_l(x - c_l) (the pull, REV = false) or p_l(x + c_l) (its transpose,
// REV = true) at site (x, y) of a row-layout state, periodic.
template <typename T, bool OFF32, bool REV>
__device__ __forceinline__ void pull9(const T* __restrict__ p, int nx, int ny, int x, int y, T (&out)[9]) {
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int yn = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  constexpr int sg = REV ? 1 : -1;
  if constexpr (OFF32) {
    const uint32_t rs = 9u * static_cast<uint32_t>(nx) * sizeof(T);
    const uint32_t rn = static_cast<uint32_t>(yn) * rs, r0 = static_cast<uint32_t>(y) * rs,
                   rp = static_cast<uint32_t>(yp) * rs;
    const uint32_t cm = static_cast<uint32_t>(xm) * sizeof(T), c0 = static_cast<uint32_t>(x) * sizeof(T),
                   cp = static_cast<uint32_t>(xp) * sizeof(T);
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      const int dx = sg * cxq(l), dy = sg * cyq(l);
      out[l] = ld_at(p + l * nx, (dy > 0 ? rp : (dy < 0 ? rn : r0)) + (dx > 0 ? cp : (dx < 0 ? cm : c0)));
    }
  } else {
    const size_t ps = static_cast<size_t>(nx), rs = 9 * ps;
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      const int dx = sg * cxq(l), dy = sg * cyq(l);
      const int xs = dx > 0 ? xp : (dx < 0 ? xm : x), ys = dy > 0 ? yp : (dy < 0 ? yn : y);
      out[l] = p[l * ps + static_cast<size_t>(ys) * rs + xs];
    }
  }
}

// store the nine values of site (x, y) of a row-layout state
template <typename T, bool OFF32>
__device__ __forceinline__ void store9(T* __restrict__ p, int nx, int x, int y, const T (&v)[9]) {
  if constexpr (OFF32) {
    const uint32_t at = static_cast<uint32_t>(y) * (9u * static_cast<uint32_t>(nx) * sizeof(T)) +
                        static_cast<uint32_t>(x) * sizeof(T);
#pragma unroll
    for (int l = 0; l < 9; ++l) st_at(p + l * nx, at, v[l]);
  } else {
    T* const out = p + static_cast<size_t>(y) * 9 * nx + x;
#pragma unroll
    for (int l = 0; l < 9; ++l) out[static_cast<size_t>(l) * nx] = v[l];
  }
}

// Sum of a workgroup's per-thread values, added to its slot (fixed order).
__device__ __forceinline__ void add_tile_sum(double v, double* slot) {
  __shared__ double sh[16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double acc = 0.0;
    const int nw = (blockDim.x * blockDim.y + 63) / 64;
    for (int w = 0; w < nw; ++w) acc += sh[w];
    *slot += acc;
  }
}

// One backward step over a tile of blockDim.x x (blockDim.y * ry) sites, one site
// per thread (the step kernel's XCD-aware tile numbering): a^t(x) from f^t pulled
// at x and a^{t+1}(x + c_l); adds the tile's sum of v . dC/dtau to its own slot of
// tau_acc.  SEED adds the loss seeds of the last two steps; OFF32 takes the
// 32-bit offset path above.
template <typename T, bool SEED, bool OFF32>
__global__ void __launch_bounds__(512) k_adj_step(const T* __restrict__ g, const T* __restrict__ ain,
                                                   T* __restrict__ aout, Seeds s, int nx, int ny,
                                                   double omega, double* tau_acc, int tiles_x, int total,
                                                   int per_xcd, int ry) {
  const int b = blockIdx.x;
  const int tile = (b & 7) * per_xcd + (b >> 3);
  if (tile >= total) return;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int x = tx * blockDim.x + threadIdx.x;
  const int ybase = (ty * blockDim.y + threadIdx.y) * ry;
  const T om = T(omega);
  double dtau = 0.0;
  if (x < nx) {
    for (int k = 0; k < ry; ++k) {
      const int y = ybase + k;
      if (y >= ny) break;
      T d[9], v[9], o[9];
      pull9<T, OFF32, false>(g, nx, ny, x, y, d);     // f^t(x - c_l)
      pull9<T, OFF32, true>(ain, nx, ny, x, y, v);    // a^{t+1}(x + c_l)
      double rh = 0.0, sx = 0.0, sy = 0.0;
      if constexpr (SEED) {
        const size_t i = static_cast<size_t>(y) * nx + x;
        rh = s.rho ? s.rho[i] : 0.0;
        sx = s.ux[i];
        sy = s.uy[i];
      }
      dtau += adjoint_site<T, SEED>(d, v, om, rh, sx, sy, o);
      store9<T, OFF32>(aout, nx, x, y, o);
    }
  }
  add_tile_sum(dtau, tau_acc + tile);
}

// Two backward steps in one launch over a tile of kA2W x TH sites: a^t from a^{t+1}
// and f^t on the tile and a one-site ring around it (kept in LDS; the neighbouring
// tiles compute the same ring values as their own), then a^{t-1} from a^t and f^{t-1}
// on the tile.  The intermediate adjoint state never leaves the CU: two steps read
// f^t, f^{t-1}, a^{t+1} and write a^{t-1}, 4 x 9 values per site instead of 6 x 9.
// Per-site arithmetic is that of k_adj_step, so a^{t-1} is the same bits as after two
// single steps; the tile's v . dC/dtau of both steps goes to its slot.  Loop counts
// are compile-time; indices past the tile's work are clamped so every load is issued
// unconditionally, and only stores and sums are guarded.
constexpr int kA2W = 64, kA2T = 256;
template <typename T, int TH, bool OFF32>
__global__ void __launch_bounds__(kA2T) k_adj_step2(const T* __restrict__ g1, const T* __restrict__ g2,
                                                    const T* __restrict__ ain, T* __restrict__ aout, int nx,
                                                    int ny, double omega, double* tau_acc, int tiles_x, int total,
                                                    int per_xcd) {
  constexpr int RW = kA2W + 2, RN = RW * (TH + 2);
  __shared__ T a1[9][RN];
  const int b = blockIdx.x;
  const int tile = (b & 7) * per_xcd + (b >> 3);
  if (tile >= total) return;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int x0 = tx * kA2W, y0 = ty * TH;
  const int tw = min(kA2W, nx - x0), th = min(TH, ny - y0);
  const int rw = tw + 2, rn = rw * (th + 2);
  const T om = T(omega);
  double dtau = 0.0;
  // the second step's f^{t-1} loads go out first: they do not depend on the first step
  constexpr int R2 = (kA2W * TH + kA2T - 1) / kA2T;
  T d2[R2][9];
#pragma unroll
  for (int k = 0; k < R2; ++k) {
    const int i = static_cast<int>(threadIdx.x) + k * kA2T;
    const int cx = min(i % kA2W, tw - 1), cyy = min(i / kA2W, th - 1);
    pull9<T, OFF32, false>(g2, nx, ny, x0 + cx, y0 + cyy, d2[k]);
  }
  // step 1 on the tile and its ring
  constexpr int R1 = (RN + kA2T - 1) / kA2T;
#pragma unroll
  for (int k = 0; k < R1; ++k) {
    const int i0 = static_cast<int>(threadIdx.x) + k * kA2T;
    const int i = min(i0, rn - 1);
    const int rx = i % rw, ry = i / rw;
    int x = x0 - 1 + rx, y = y0 - 1 + ry;
    x += x < 0 ? nx : 0;
    x -= x >= nx ? nx : 0;
    y += y < 0 ? ny : 0;
    y -= y >= ny ? ny : 0;
    T d[9], v[9], o[9];
    pull9<T, OFF32, false>(g1, nx, ny, x, y, d);
    pull9<T, OFF32, true>(ain, nx, ny, x, y, v);
    const double nq = adjoint_site<T, false>(d, v, om, 0.0, 0.0, 0.0, o);
    if (i0 < rn) {
#pragma unroll
      for (int l = 0; l < 9; ++l) a1[l][ry * RW + rx] = o[l];
      if (rx >= 1 && rx <= tw && ry >= 1 && ry <= th) dtau += nq;
    }
  }
  __syncthreads();
  // step 2 on the tile: v_l = a^t_l(x + c_l) from the LDS copy
#pragma unroll
  for (int k = 0; k < R2; ++k) {
    const int i = static_cast<int>(threadIdx.x) + k * kA2T;
    const int lx = i % kA2W, ly = i / kA2W;
    const bool live = lx < tw && ly < th;
    const int cx = min(lx, tw - 1), cyy = min(ly, th - 1);
    const int x = x0 + cx, y = y0 + cyy;
    T v[9], o[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) v[l] = a1[l][(cyy + 1 + cyq(l)) * RW + (cx + 1 + cxq(l))];
    const double nq = adjoint_site<T, false>(d2[k], v, om, 0.0, 0.0, 0.0, o);
    if (live) {
      store9<T, OFF32>(aout, nx, x, y, o);
      dtau += nq;
    }
  }
  add_tile_sum(dtau, tau_acc + tile);
}

// du0 = sum_l a^0_l df^eq_l/du at (rho0 = 1, u0)
template <typename T>
__global__ void __launch_bounds__(kAT) k_adj_u0(const T* __restrict__ adj, const double* __restrict__ ux0,
                                                const double* __restrict__ uy0, PopLayout lay, int nx,
                                                int ny, double* gx, double* gy) {
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t i = blockIdx.x * size_t(kAT) + threadIdx.x;
  if (i >= plane) return;
  const double ux = ux0[i], uy = uy0[i];
  const size_t at = (i / nx) * lay.rs + (i % nx);
  double bx = 0.0, by = 0.0;
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const double a = double(adj[l * lay.ps + at]);
    const double cu = cxq(l) * ux + cyq(l) * uy;
    bx += a * wq(l) * (3.0 * cxq(l) + 9.0 * cu * cxq(l) - 3.0 * ux);
    by += a * wq(l) * (3.0 * cyq(l) + 9.0 * cu * cyq(l) - 3.0 * uy);
  }
  gx[i] = bx;
  gy[i] = by;
}

__global__ void k_zero(double* p, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

// ---- workspace ------------------------------------------------------------------------
struct AdjWs {
  void* ckpt;          // [nck][9][plane] storage type
  void* seg[2];        // [K+1][9][plane] each; the second only with two or more segments
  void* adj[2];        // [9][plane]
  double* mom[3][3];   // levels T-2, T-1, T: rho, ux, uy
  double* r;           // residual field
  double* rmap;        // window means R(corner)
  double* rhat;
  double* w;           // [kAdjFields][plane]
  double* small;       // scalars / partials
  double* tau_acc;     // [blocks]
  double* fill;        // zero field for rho0... (rho0 = 1 field)
  BalanceWs bal;
  size_t bytes;
};

int nblocks_sites(size_t plane) { return static_cast<int>((plane + kAT - 1) / kAT); }

// second: a second segment buffer (the backward's recomputation then runs ahead on its own stream)
AdjWs carve_adj(const lbm_adjoint_config& c, void* base, size_t cap, bool second = true) {
  Carver cv(base, cap);
  const size_t plane = static_cast<size_t>(c.nx) * c.ny;
  const size_t es = c.dtype == LBM_F32 ? 4 : 8;
  const int64_t nck = (c.steps + c.ckpt_every - 1) / c.ckpt_every;
  AdjWs w{};
  w.ckpt = cv.take<char>(static_cast<size_t>(nck) * 9 * plane * es);
  const size_t seg_bytes = static_cast<size_t>(c.ckpt_every + 1) * 9 * plane * es;
  w.seg[0] = cv.take<char>(seg_bytes);
  w.seg[1] = (second && nck > 1) ? cv.take<char>(seg_bytes) : w.seg[0];
  w.adj[0] = cv.take<char>(9 * plane * es);
  w.adj[1] = cv.take<char>(9 * plane * es);
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < 3; ++k) w.mom[l][k] = cv.take<double>(plane);
  w.r = cv.take<double>(plane);
  w.rmap = cv.take<double>(plane);
  w.rhat = cv.take<double>(plane);
  w.w = cv.take<double>(static_cast<size_t>(kAdjFields) * plane);
  w.small = cv.take<double>(4096 + 64);
  // one slot per tile of the launch shape; a tile holds >= 64 threads, so this bounds any shape
  w.tau_acc = cv.take<double>(std::max<size_t>(plane / 16, static_cast<size_t>(c.ny)) + 1024);
  w.fill = cv.take<double>(plane);
  w.bal = carve_balance(cv, c.nx, c.ny);
  w.bytes = cv.used + 256;
  return w;
}

int validate_adj(const lbm_adjoint_config* c) {
  if (!c) return fail(LBM_E_INVALID, "config is NULL");
  if (c->nx < 16 || c->ny < 16 || c->nx > 16384 || c->ny > 16384)
    return fail(LBM_E_INVALID, "grid %d x %d outside [16, 16384]", c->nx, c->ny);
  if (c->dtype != LBM_F32 && c->dtype != LBM_F64) return fail(LBM_E_INVALID, "bad dtype");
  if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return fail(LBM_E_INVALID, "tau must be > 0.5");
  if (c->steps < 2 || c->steps > 10000000) return fail(LBM_E_INVALID, "steps must be >= 2");
  if (c->ckpt_every < 1 || c->ckpt_every > 100000) return fail(LBM_E_INVALID, "ckpt_every >= 1");
  const int m = std::min(c->nx, c->ny);
  if (c->box < 1 || c->box > m) return fail(LBM_E_INVALID, "box %d outside [1, %d]", c->box, m);
  if (c->reserved != 0) return fail(LBM_E_INVALID, "reserved must be 0");
  return LBM_OK;
}

constexpr int kAdjLayout = LBM_LAYOUT_ROWS;

template <typename T>
int launch_adj_init(const void* g, void* adj, Seeds s, int nx, int ny, hipStream_t st) {
  const size_t plane = static_cast<size_t>(nx) * ny;
  hipLaunchKernelGGL(k_adj_init<T>, dim3(nblocks_sites(plane)), dim3(kAT), 0, st,
                     static_cast<const T*>(g), static_cast<T*>(adj), s,
                     pop_layout(kAdjLayout, nx, ny), nx, ny);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

// One backward step in the launch shape t (its bx, by and ry; one site per thread).
template <typename T>
int launch_adj_step(const void* g, const void* ain, void* aout, Seeds s, int has_seed, int nx, int ny,
                    double omega, double* tau_acc, const lbm_tile& t, hipStream_t st) {
  const int tiles_x = (nx + t.bx - 1) / t.bx;
  const int tiles_y = (ny + t.by * t.ry - 1) / (t.by * t.ry);
  const int total = tiles_x * tiles_y;
  const int per_xcd = (total + 7) / 8;
  const bool off32 = 9ull * static_cast<uint64_t>(nx) * ny * sizeof(T) <= 0xffffffffull;
  auto kern = has_seed ? (off32 ? k_adj_step<T, true, true> : k_adj_step<T, true, false>)
                       : (off32 ? k_adj_step<T, false, true> : k_adj_step<T, false, false>);
  hipLaunchKernelGGL(kern, dim3(per_xcd * 8), dim3(t.bx, t.by), 0, st, static_cast<const T*>(g),
                     static_cast<const T*>(ain), static_cast<T*>(aout), s, nx, ny, omega, tau_acc, tiles_x,
                     total, per_xcd, t.ry);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

// Band height of the two-step kernel: 16 rows in FP32 when that still gives 1024
// tiles (42.8 KiB of LDS), else 8 (23.8 KiB in FP32, 47.5 KiB in FP64).
template <typename T>
int pair_rows(int nx, int ny) {
  const int tx = (nx + kA2W - 1) / kA2W;
  return (sizeof(T) == 4 && tx * ((ny + 15) / 16) >= 1024) ? 16 : 8;
}
template <typename T>
int pair_tiles(int nx, int ny) {
  const int th = pair_rows<T>(nx, ny);
  return ((nx + kA2W - 1) / kA2W) * ((ny + th - 1) / th);
}

// Two backward steps: a^{t-1} (aout) from a^{t+1} (ain), g1 = f^t and g2 = f^{t-1}.
template <typename T>
int launch_adj_pair(const void* g1, const void* g2, const void* ain, void* aout, int nx, int ny,
                    double omega, double* tau_acc, hipStream_t st) {
  const int th = pair_rows<T>(nx, ny);
  const int tiles_x = (nx + kA2W - 1) / kA2W;
  const int total = tiles_x * ((ny + th - 1) / th);
  const int per_xcd = (total + 7) / 8;
  const bool off32 = 9ull * static_cast<uint64_t>(nx) * ny * sizeof(T) <= 0xffffffffull;
  auto kern = th == 16 ? (off32 ? k_adj_step2<T, 16, true> : k_adj_step2<T, 16, false>)
                       : (off32 ? k_adj_step2<T, 8, true> : k_adj_step2<T, 8, false>);
  hipLaunchKernelGGL(kern, dim3(per_xcd * 8), dim3(kA2T), 0, st, static_cast<const T*>(g1),
                     static_cast<const T*>(g2), static_cast<const T*>(ain), static_cast<T*>(aout), nx, ny,
                     omega, tau_acc, tiles_x, total, per_xcd);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

// number of tiles of a launch shape (slots of the tau accumulator)
int tile_count(int nx, int ny, const lbm_tile& t) {
  return ((nx + t.bx - 1) / t.bx) * ((ny + t.by * t.ry - 1) / (t.by * t.ry));
}

template <typename T>
int launch_adj_u0(const void* adj, const double* ux0, const double* uy0, int nx, int ny,
                  double* gx, double* gy, hipStream_t st) {
  const size_t plane = static_cast<size_t>(nx) * ny;
  hipLaunchKernelGGL(k_adj_u0<T>, dim3(nblocks_sites(plane)), dim3(kAT), 0, st,
                     static_cast<const T*>(adj), ux0, uy0, pop_layout(kAdjLayout, nx, ny), nx, ny, gx,
                     gy);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

struct Runner {
  lbm_adjoint_config c;
  AdjWs w;
  hipStream_t s;
  size_t plane, state_bytes;
  lbm_tile tile;   // single-step shape (the segments keep every intermediate state)
  lbm_tile ftile;  // shape of the first forward pass, which keeps only checkpoints
  void* seg_state(int b, int k) const { return static_cast<char*>(w.seg[b]) + k * state_bytes; }
  void* ckpt_state(int64_t k) const { return static_cast<char*>(w.ckpt) + k * state_bytes; }

  int step(const void* src, void* dst, double* hr, double* hx, double* hy) {
    return step_on(s, src, dst, hr, hx, hy);
  }
  int step_on(hipStream_t st, const void* src, void* dst, double* hr, double* hx, double* hy,
              bool multi = false) {
    StepParams p{};
    p.src = src;
    p.dst = dst;
    p.h_rho = hr;
    p.h_ux = hx;
    p.h_uy = hy;
    p.nx = c.nx;
    p.ny = c.ny;
    const PopLayout lay = pop_layout(kAdjLayout, c.nx, c.ny);
    p.ps = lay.ps;
    p.rs = lay.rs;
    p.omega = 1.0 / c.tau;
    p.alpha = 0.0;
    return launch_step(c.dtype, false, p, multi ? ftile : tile, st);
  }
};

// Graphs captured on a private stream, destroyed with the cache, and the
// second stream on which the backward pass recomputes the next segment.
struct GraphCache {
  hipStream_t cs = nullptr;
  hipStream_t main = nullptr;   // replays go here; synchronised before the graphs are freed
  hipStream_t rs = nullptr;     // recomputation stream (default priority, like every stream here)
  hipEvent_t go = nullptr, fwd_done[2] = {nullptr, nullptr}, bwd_done[2] = {nullptr, nullptr};
  hipGraphExec_t fwd[2] = {nullptr, nullptr};   // K steps through segment buffer b
  hipGraphExec_t ffwd = nullptr;  // first pass: K steps, intermediate states not kept
  // [adjoint parity][buffer][parity of the segment's first step], with its launch count
  hipGraphExec_t bwd[2][2][2] = {};
  int bwd_launches[2][2][2] = {};
  int init() {
    LBM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    LBM_HIP(hipStreamCreateWithFlags(&rs, hipStreamNonBlocking));
    LBM_HIP(hipEventCreateWithFlags(&go, hipEventDisableTiming));
    for (int b = 0; b < 2; ++b) {
      LBM_HIP(hipEventCreateWithFlags(&fwd_done[b], hipEventDisableTiming));
      LBM_HIP(hipEventCreateWithFlags(&bwd_done[b], hipEventDisableTiming));
    }
    return LBM_OK;
  }
  template <class F>
  int capture(hipGraphExec_t* out, F&& body) {
    hipGraph_t g = nullptr;
    LBM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const int rc = body(cs);
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc != LBM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return LBM_OK;
  }
  ~GraphCache() {
    if (main) (void)hipStreamSynchronize(main);
    if (rs) (void)hipStreamSynchronize(rs);
    for (auto& f : fwd)
      if (f) (void)hipGraphExecDestroy(f);
    if (ffwd) (void)hipGraphExecDestroy(ffwd);
    for (auto& bp : bwd)
      for (auto& bb : bp)
        for (auto& b : bb)
          if (b) (void)hipGraphExecDestroy(b);
    for (hipEvent_t e : {go, fwd_done[0], fwd_done[1], bwd_done[0], bwd_done[1]})
      if (e) (void)hipEventDestroy(e);
    if (rs) (void)hipStreamDestroy(rs);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" {

int lbm_adjoint_workspace_bytes(const lbm_adjoint_config* cfg, size_t* bytes) {
  if (int rc = validate_adj(cfg)) return rc;
  if (!bytes) return fail(LBM_E_INVALID, "bytes is NULL");
  *bytes = carve_adj(*cfg, nullptr, 0).bytes;
  return LBM_OK;
}

int lbm_adjoint_run(const lbm_adjoint_config* cfg, void* ws, size_t ws_bytes, const double* ux0,
                    const double* uy0, double* loss, double* grad_ux0, double* grad_uy0,
                    double* grad_tau) {
  if (int rc = validate_adj(cfg)) return rc;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(LBM_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
  if (!ux0 || !uy0 || !loss) return fail(LBM_E_INVALID, "ux0, uy0 and loss must not be NULL");
  if ((grad_ux0 == nullptr) != (grad_uy0 == nullptr))
    return fail(LBM_E_INVALID, "grad_ux0 and grad_uy0 must both be given or both be NULL");
  // the preferred size holds two segment buffers; one is enough, without the overlap
  const size_t need = carve_adj(*cfg, nullptr, 0, false).bytes;
  const bool two = ws_bytes >= carve_adj(*cfg, nullptr, 0, true).bytes;
  if (ws_bytes < need) return fail(LBM_E_NOMEM, "workspace %zu < %zu", ws_bytes, need);

  Runner R;
  R.c = *cfg;
  R.w = carve_adj(*cfg, ws, ws_bytes, two);
  R.s = static_cast<hipStream_t>(cfg->stream);
  R.plane = static_cast<size_t>(cfg->nx) * cfg->ny;
  R.state_bytes = 9 * R.plane * (cfg->dtype == LBM_F32 ? 4 : 8);
  // the single-step shape tuned for this grid if lbm_autotune has seen it, else the default
  // (the segments keep every intermediate state, so each launch advances one step)
  // and, for the first forward pass, the tuned shape whatever its steps per launch
  lbm_tile tuned{};
  const bool have_tuned = tuned_tile(cfg->dtype, cfg->nx, cfg->ny, false, kAdjLayout, &tuned);
  R.tile = (have_tuned && steps_per_launch(tuned) == 1)
               ? tuned
               : default_tile(cfg->dtype, cfg->nx, cfg->ny, kAdjLayout);
  R.ftile = have_tuned ? tuned : R.tile;
  // the recomputed states and the adjoint fields are read again within a few
  // launches: keep their stores cacheable
  R.tile.nt = 0;
  const int nx = cfg->nx, ny = cfg->ny;
  const int64_t T = cfg->steps;
  const int K = cfg->ckpt_every;
  const hipStream_t s = R.s;
  const int g = static_cast<int>(std::min<size_t>((R.plane + 255) / 256, 4096));

  // ---- forward: init, steps with checkpoints, moments at T-2, T-1, T ----
  hipLaunchKernelGGL(k_set, dim3(g), dim3(256), 0, s, R.w.fill, R.plane, 1.0);   // rho0 = 1
  LBM_HIP(hipGetLastError());
  if (int rc = launch_init(cfg->dtype, R.ckpt_state(0), pop_layout(kAdjLayout, nx, ny), R.w.fill,
                           ux0, uy0, nx, ny, s))
    return rc;
  // Full segments without a recorded level replay captured graphs of K steps
  // through the segment buffer (seg[0] -> seg[K]); the rest is launched directly.
  const int64_t nseg = (T + K - 1) / K;
  GraphCache gc;
  gc.main = s;
  if (int rc = gc.init()) return rc;
  auto seg_len = [&](int64_t sg) { return std::min<int64_t>(sg * K + K, T) - sg * K; };
  auto seg_plain = [&](int64_t sg) { return seg_len(sg) == K && sg * K + K <= T - 2; };
  // segment sg from its checkpoint through segment buffer b on stream st
  auto forward_segment = [&](int64_t sg, bool record, int b, hipStream_t st) -> int {
    const int64_t t0 = sg * K, len = seg_len(sg);
    LBM_HIP(hipMemcpyAsync(R.seg_state(b, 0), R.ckpt_state(sg), R.state_bytes, hipMemcpyDeviceToDevice, st));
    if (seg_plain(sg)) {
      if (!gc.fwd[b]) {
        if (int rc = gc.capture(&gc.fwd[b], [&](hipStream_t cs) -> int {
              for (int k = 0; k < K; ++k)
                if (int r2 = R.step_on(cs, R.seg_state(b, k), R.seg_state(b, k + 1), nullptr, nullptr, nullptr))
                  return r2;
              return LBM_OK;
            }))
          return rc;
      }
      LBM_HIP(hipGraphLaunch(gc.fwd[b], st));
      return LBM_OK;
    }
    for (int64_t k = 0; k < len; ++k) {
      const int64_t t = t0 + k;
      double* h[3] = {nullptr, nullptr, nullptr};
      if (record && (t == T - 2 || t == T - 1)) {
        const int lv = static_cast<int>(t - (T - 2));
        for (int q = 0; q < 3; ++q) h[q] = R.w.mom[lv][q];
      }
      if (int rc = R.step_on(st, R.seg_state(b, static_cast<int>(k)), R.seg_state(b, static_cast<int>(k + 1)),
                             h[0], h[1], h[2]))
        return rc;
    }
    return LBM_OK;
  };
  // First pass over a full segment: only its end state is kept (the next
  // checkpoint), so it runs in the tuned shape, possibly several steps per
  // launch, ping-ponging between seg[0] and seg[1]; returns the final buffer.
  const int spl = steps_per_launch(R.ftile);
  const int ff_par = (K / spl + K % spl) & 1;
  auto fast_segment = [&](int64_t sg) -> int {
    LBM_HIP(hipMemcpyAsync(R.seg_state(0, 0), R.ckpt_state(sg), R.state_bytes, hipMemcpyDeviceToDevice, s));
    if (!gc.ffwd) {
      if (int rc = gc.capture(&gc.ffwd, [&](hipStream_t cs) -> int {
            int p = 0;
            for (int k = 0; k + spl <= K; k += spl, p ^= 1)
              if (int r2 = R.step_on(cs, R.seg_state(0, p), R.seg_state(0, p ^ 1), nullptr, nullptr, nullptr, true))
                return r2;
            for (int k = 0; k < K % spl; ++k, p ^= 1)
              if (int r2 = R.step_on(cs, R.seg_state(0, p), R.seg_state(0, p ^ 1), nullptr, nullptr, nullptr))
                return r2;
            return LBM_OK;
          }))
        return rc;
    }
    LBM_HIP(hipGraphLaunch(gc.ffwd, s));
    return LBM_OK;
  };
  for (int64_t sg = 0; sg < nseg; ++sg) {
    if (seg_plain(sg) && sg + 1 < nseg) {
      if (int rc = fast_segment(sg)) return rc;
      LBM_HIP(hipMemcpyAsync(R.ckpt_state(sg + 1), R.seg_state(0, ff_par), R.state_bytes,
                             hipMemcpyDeviceToDevice, s));
      continue;
    }
    if (int rc = forward_segment(sg, true, 0, s)) return rc;
    if (sg + 1 < nseg)
      LBM_HIP(hipMemcpyAsync(R.ckpt_state(sg + 1), R.seg_state(0, static_cast<int>(seg_len(sg))),
                             R.state_bytes, hipMemcpyDeviceToDevice, s));
  }
  void* cur = R.seg_state(0, static_cast<int>(seg_len(nseg - 1)));   // g^T
  {
    MomentParams m{};
    m.pop = cur;
    m.out_dtype = LBM_F64;
    m.rho64 = R.w.mom[2][0];
    m.ux64 = R.w.mom[2][1];
    m.uy64 = R.w.mom[2][2];
    m.partials = R.w.w;  // scratch (block partials, overwritten later)
    m.nx = nx;
    m.ny = ny;
    m.ps = pop_layout(kAdjLayout, nx, ny).ps;
    m.rs = pop_layout(kAdjLayout, nx, ny).rs;
    if (int rc = launch_moments(cfg->dtype, false, m, s)) return rc;
  }

  // ---- loss ----
  lbm_balance_input in{};
  in.nx = nx;
  in.ny = ny;
  in.nu = (cfg->tau - 0.5) / 3.0;
  for (int l = 0; l < 3; ++l) {
    in.rho[l] = R.w.mom[l][0];
    in.ux[l] = R.w.mom[l][1];
    in.uy[l] = R.w.mom[l][2];
  }
  in.stream = s;
  if (int rc = balance_terms(in, R.w.bal)) return rc;
  hipLaunchKernelGGL(k_residual, dim3(g), dim3(256), 0, s, R.w.bal.terms, R.plane, R.w.r);
  LBM_HIP(hipGetLastError());
  const int L = cfg->box;
  const bool single = (L == nx && L == ny);
  double* rmean = R.w.small + 4096 + 8;
  double* part = R.w.small;   // up to 4096 partials
  if (int rc = field_means(R.w.r, 1, nx, ny, R.w.bal.partials + R.w.bal.partials_cap, rmean, s)) return rc;
  double* jdev = R.w.small + 4096 + 16;
  const double nwin = single ? 1.0 : double(R.plane);
  if (single) {
    // J = mean(r)^2; dJ/dr = 2 mean(r) / N^2
    hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(256), 0, s, rmean, static_cast<size_t>(1), part);
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, 1, 1.0, jdev);
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fill, dim3(g), dim3(256), 0, s, R.w.rhat, R.plane, rmean,
                       2.0 / double(R.plane));
    LBM_HIP(hipGetLastError());
  } else {
    double* sat = R.w.bal.sat;
    if (int rc = sat_build(R.w.r, 1, rmean, sat, nx, ny, s)) return rc;
    if (int rc = box_map(sat, rmean, 1, 0, L, 0, 1.0 / (double(L) * L), R.w.rmap, nx, ny, s)) return rc;
    hipLaunchKernelGGL(k_sumsq, dim3(g), dim3(256), 0, s, R.w.rmap, R.plane, part);
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, g, 1.0 / nwin, jdev);
    LBM_HIP(hipGetLastError());
    // dJ/dr(x) = 2/(W L^2) * sum of R over the corners whose window holds x
    double* rmm = R.w.small + 4096 + 24;
    if (int rc = field_means(R.w.rmap, 1, nx, ny, R.w.bal.partials + R.w.bal.partials_cap, rmm, s))
      return rc;
    if (int rc = sat_build(R.w.rmap, 1, rmm, sat, nx, ny, s)) return rc;
    if (int rc = box_map(sat, rmm, 1, 0, L, -(L - 1), 2.0 / (nwin * double(L) * L), R.w.rhat, nx, ny, s))
      return rc;
  }
  LBM_HIP(hipMemcpyAsync(loss, jdev, sizeof(double), hipMemcpyDeviceToHost, s));
  if (!grad_ux0 && !grad_tau) {
    LBM_HIP(hipStreamSynchronize(s));
    return LBM_OK;
  }

  // The backward pass sweeps segment sg from buffer (nseg - 1 - sg) % nbuf (the last
  // segment's states are still in buffer 0 from the forward pass) while, with two
  // buffers, the second stream recomputes segment sg - 1 into the other buffer from its
  // checkpoint.  A recomputation waits for the sweep that last read its buffer (with one
  // buffer: the sweep just before it); a sweep waits for its recomputation.  Kernels and
  // operands are those of a one-stream run.
  const int nbuf = (two && nseg > 1) ? 2 : 1;
  auto buf_of = [&](int64_t sg) { return static_cast<int>((nseg - 1 - sg) % nbuf); };
  auto recompute = [&](int64_t sg) -> int {
    const int b = buf_of(sg);
    if (sg + nbuf <= nseg - 1) LBM_HIP(hipStreamWaitEvent(gc.rs, gc.bwd_done[b], 0));
    if (int rc = forward_segment(sg, false, b, gc.rs)) return rc;
    LBM_HIP(hipEventRecord(gc.fwd_done[b], gc.rs));
    return LBM_OK;
  };
  if (nbuf == 2) {
    // checkpoints are complete once the forward pass's work on s is
    LBM_HIP(hipEventRecord(gc.go, s));
    LBM_HIP(hipStreamWaitEvent(gc.rs, gc.go, 0));
    if (int rc = recompute(nseg - 2)) return rc;
  }

  // ---- loss adjoint: seeds at T, T-1, T-2 and the explicit nu derivative ----
  AdjLoss al{};
  al.rho = R.w.mom[2][0];
  al.ux = R.w.mom[2][1];
  al.uy = R.w.mom[2][2];
  al.ux1 = R.w.mom[1][1];
  al.uy1 = R.w.mom[1][2];
  al.ux2 = R.w.mom[0][1];
  al.uy2 = R.w.mom[0][2];
  al.aux = R.w.bal.aux;
  al.rhat = R.w.rhat;
  al.w = R.w.w;
  al.nu = in.nu;
  al.nx = nx;
  al.ny = ny;
  dim3 blk(64, 4), grd((nx + 63) / 64, (ny + 3) / 4);
  hipLaunchKernelGGL(k_loss_b1, grd, blk, 0, s, al);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_loss_b2, grd, blk, 0, s, al);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_loss_b3, grd, blk, 0, s, al);
  LBM_HIP(hipGetLastError());
  double* nuh = R.w.small + 4096 + 32;
  hipLaunchKernelGGL(k_sum, dim3(g), dim3(256), 0, s, R.w.w + S_NUS * R.plane, R.plane, part);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, g, 1.0, nuh);
  LBM_HIP(hipGetLastError());

  // ---- population adjoint, segment by segment from the last ----
  // slots of the single-step and the two-step tilings (both add into tau_acc)
  // The adjoint steps take a fixed shape (not the tuned one), so the slots' partial sums
  // of dJ/dtau, and thus its bits, do not depend on the step kernel's tuning.
  const lbm_tile atile = default_tile(cfg->dtype, nx, ny, kAdjLayout);
  const int nb = std::max(tile_count(nx, ny, atile), cfg->dtype == LBM_F32 ? pair_tiles<float>(nx, ny)
                                                                           : pair_tiles<double>(nx, ny));
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, R.w.tau_acc, static_cast<size_t>(nb));
  LBM_HIP(hipGetLastError());
  const double omega = 1.0 / cfg->tau;
  const Seeds sT{R.w.w + S_RHON * R.plane, R.w.w + S_UXN * R.plane, R.w.w + S_UYN * R.plane};
  const Seeds s1{nullptr, R.w.w + S_UX1 * R.plane, R.w.w + S_UY1 * R.plane};
  const Seeds s2{nullptr, R.w.w + S_UX2 * R.plane, R.w.w + S_UY2 * R.plane};
  const bool f32 = cfg->dtype == LBM_F32;
  int par = 0;                       // ain = adj[par], aout = adj[par ^ 1]
  for (int64_t sg = nseg - 1; sg >= 0; --sg) {
    const int64_t t0 = sg * K;
    const int64_t t1 = t0 + seg_len(sg);
    const int b = buf_of(sg);
    if (sg != nseg - 1) LBM_HIP(hipStreamWaitEvent(s, gc.fwd_done[b], 0));
    if (sg == nseg - 1) {
      const void* gT = R.seg_state(b, static_cast<int>(t1 - t0));
      const int rc = f32 ? launch_adj_init<float>(gT, R.w.adj[par], sT, nx, ny, s)
                         : launch_adj_init<double>(gT, R.w.adj[par], sT, nx, ny, s);
      if (rc) return rc;
    }
    const bool seeded = t1 >= T - 1;   // holds t = T-1 or T-2
    // Steps t and t - 1 go in one two-step launch when t is odd and neither is seeded
    // (pairs fall on the same steps whatever the checkpoint interval); the rest run
    // one step per launch.  *n receives the number of launches (each flips the buffers).
    auto sweep = [&](hipStream_t st, int pp, int* n) -> int {
      *n = 0;
      for (int64_t t = t1 - 1; t >= t0; ++*n, pp ^= 1) {
        const bool seed = (t == T - 1) || (t == T - 2);
        const void* gt = R.seg_state(b, static_cast<int>(t - t0));
        int rc;
        if (!seed && (t & 1) && t - 1 >= t0) {
          const void* gp = R.seg_state(b, static_cast<int>(t - 1 - t0));
          rc = f32 ? launch_adj_pair<float>(gt, gp, R.w.adj[pp], R.w.adj[pp ^ 1], nx, ny, omega, R.w.tau_acc, st)
                   : launch_adj_pair<double>(gt, gp, R.w.adj[pp], R.w.adj[pp ^ 1], nx, ny, omega, R.w.tau_acc, st);
          t -= 2;
        } else {
          const Seeds sd = (t == T - 1) ? s1 : s2;
          rc = f32 ? launch_adj_step<float>(gt, R.w.adj[pp], R.w.adj[pp ^ 1], sd, seed ? 1 : 0, nx, ny, omega,
                                            R.w.tau_acc, atile, st)
                   : launch_adj_step<double>(gt, R.w.adj[pp], R.w.adj[pp ^ 1], sd, seed ? 1 : 0, nx, ny, omega,
                                             R.w.tau_acc, atile, st);
          t -= 1;
        }
        if (rc) return rc;
      }
      return LBM_OK;
    };
    if (seg_len(sg) == K && !seeded) {
      const int tp = static_cast<int>(t0 & 1);
      hipGraphExec_t& gb = gc.bwd[par][b][tp];
      if (!gb) {
        const int p0 = par;
        int& nl = gc.bwd_launches[par][b][tp];
        if (int rc = gc.capture(&gb, [&](hipStream_t cs) -> int { return sweep(cs, p0, &nl); }))
          return rc;
      }
      LBM_HIP(hipGraphLaunch(gb, s));
      par ^= gc.bwd_launches[par][b][tp] & 1;
    } else {
      int n = 0;
      if (int rc = sweep(s, par, &n)) return rc;
      par ^= n & 1;
    }
    if (sg >= nbuf) {
      LBM_HIP(hipEventRecord(gc.bwd_done[b], s));
      if (int rc = recompute(sg - nbuf)) return rc;
    }
  }
  void* ain = R.w.adj[par];
  // ain now holds dJ/df^0
  if (grad_ux0) {
    const int rc = f32 ? launch_adj_u0<float>(ain, ux0, uy0, nx, ny, grad_ux0, grad_uy0, s)
                       : launch_adj_u0<double>(ain, ux0, uy0, nx, ny, grad_ux0, grad_uy0, s);
    if (rc) return rc;
  }
  double tsum_dev_host[2] = {0.0, 0.0};
  double* tsum = R.w.small + 4096 + 40;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, R.w.tau_acc, nb, 1.0, tsum);
  LBM_HIP(hipGetLastError());
  LBM_HIP(hipMemcpyAsync(&tsum_dev_host[0], tsum, sizeof(double), hipMemcpyDeviceToHost, s));
  LBM_HIP(hipMemcpyAsync(&tsum_dev_host[1], nuh, sizeof(double), hipMemcpyDeviceToHost, s));
  LBM_HIP(hipStreamSynchronize(s));
  // dJ/dtau = collision part + explicit viscosity part (dnu/dtau = 1/3)
  if (grad_tau) *grad_tau = tsum_dev_host[0] + tsum_dev_host[1] / 3.0;
  return LBM_OK;
}

}  // extern "C"
