// Sub-volume energy / enstrophy balance on gfx950 (FP64 throughout).
//
//   pass A  : pointwise terms and the level-n fields needed by later passes
//             (8th-order centred differences of Eq. 18, three-level time
//             derivative of Eq. 17)
//   pass B  : terms that difference products of pass-A fields
//   pass C  : the diffusion term of the enstrophy balance (third composed
//             difference, total stencil radius 12)
//             (passes A-C on two sites per thread with 16-byte loads where the
//             width is even and the fields aligned, bitwise the same results)
//   means   : domain mean of each of the 13 fields (deterministic two-level sum
//             of the passes' workgroup sums)
//   SAT     : mean-centred inclusive 2D prefix sums, one (ny+1) x (nx+1) table
//             per field, rows of all fields at one y adjacent and 128-byte
//             aligned.  The two-site passes write their rows as 128-site scans
//             straight into the table; a column pass adds each row's carry from
//             the tiles to its left, centres on the mean and scans the columns
//             (the table is read and written once after the passes).  The
//             one-site passes write term planes, scanned by a row pass first.
//   windows : for each box side L and every window corner, the 13 box means
//             (differences of the table across the window's top and bottom
//             rows, periodic wrap through the table totals), the balancing
//             errors of Eqs. 12-13 and the Mach number of Eq. 20, reduced to
//             count / sum / sum of squares / min / max / NaN per block and
//             merged in a fixed order.  Corners are visited along sequences
//             y0, y0 + L, y0 + 2L, ... so a window's bottom row is the next
//             window's top row and each table row is read once per side; a
//             side L and its double 2L share one walk when both are asked for.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "lbm_fd8.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

using namespace fd8;

constexpr int NT = LBM_NTERMS;
enum { A_E = 0, A_OM2 = 1, A_W = 2, A_SXX = 3, A_SYY = 4, A_SXY = 5, A_HX = 6, A_HY = 7, NAUX = 8 };

struct PassArgs {
  const double* rho[3];
  const double* ux[3];
  const double* uy[3];
  const double* fx;
  const double* fy;
  double nu;
  const double* nu_field;  // per-site viscosity at level n, or null
  int nx, ny;
  double* terms;  // [13][ny][nx] term fields, or null (paired passes writing the table only)
  double* aux;
  double* psum;  // paired passes: [13][blocks] workgroup sums of each term field
  // paired passes, when non-null: each wave's 128 sites of a row, scanned, as
  // entries x + 1 of the prefix table's rows y + 1 (rows ld doubles apart), and
  // the 128-site totals in rtot[(y * 13 + field) * gridDim.x + blockIdx.x]
  double* sat;
  double* rtot;
  int ld;
};

// Weights of Eq. 18 per offset m = 1..4 (the difference g(i+m) - g(i-m) is
// multiplied by kFd8[m-1]); each stencil below accumulates over m in a loop
// that is not unrolled, so that only one offset's loads are live at a time.
__constant__ double kFd8[4] = {4.0 / 5.0, -1.0 / 5.0, (4.0 / 21.0) / 5.0, -(1.0 / 56.0) / 5.0};

__global__ void __launch_bounds__(256) k_bal_a(PassArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const int nx = a.nx, ny = a.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t i = static_cast<size_t>(y) * nx + x;
  // d_x u_y and d_y u_x at the three levels; d_x u_x, d_y u_y, grad rho at level n
  double dxuy[3] = {0.0, 0.0, 0.0}, dyux[3] = {0.0, 0.0, 0.0};
  double dxux = 0.0, dyuy = 0.0, dxr = 0.0, dyr = 0.0;
#pragma unroll 1
  for (int m = 1; m <= 4; ++m) {
    const double c = kFd8[m - 1];
    const size_t xp = static_cast<size_t>(y) * nx + wrap_add(x, m, nx);
    const size_t xm = static_cast<size_t>(y) * nx + wrap_add(x, -m, nx);
    const size_t yp = static_cast<size_t>(wrap_add(y, m, ny)) * nx + x;
    const size_t ym = static_cast<size_t>(wrap_add(y, -m, ny)) * nx + x;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dxuy[k] += c * (a.uy[k][xp] - a.uy[k][xm]);
      dyux[k] += c * (a.ux[k][yp] - a.ux[k][ym]);
    }
    dxux += c * (a.ux[2][xp] - a.ux[2][xm]);
    dyuy += c * (a.uy[2][yp] - a.uy[2][ym]);
    dxr += c * (a.rho[2][xp] - a.rho[2][xm]);
    dyr += c * (a.rho[2][yp] - a.rho[2][ym]);
  }
  double om[3], en[3], ens[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    om[k] = dxuy[k] - dyux[k];
    ens[k] = 0.5 * om[k] * om[k];
    const double vx = a.ux[k][i], vy = a.uy[k][i];
    en[k] = 0.5 * a.rho[k][i] * (vx * vx + vy * vy);
  }
  const double dyux_n = dyux[2], dxuy_n = dxuy[2];
  const double r = a.rho[2][i], vx = a.ux[2][i], vy = a.uy[2][i];
  const double dxp = dxr / 3.0;
  const double dyp = dyr / 3.0;
  const double nu = a.nu_field ? a.nu_field[i] : a.nu;
  const double sxx = 2.0 * nu * r * dxux;
  const double syy = 2.0 * nu * r * dyuy;
  const double sxy = nu * r * (dxuy_n + dyux_n);
  double fxv = 0.0, fyv = 0.0;
  if (a.fx) {
    fxv = a.fx[i];
    fyv = a.fy[i];
  }
  double* t = a.terms;
  t[LBM_T_LHS_E * plane + i] = (3.0 * en[2] - 4.0 * en[1] + en[0]) / 2.0;
  t[LBM_T_E2 * plane + i] = -(vx * dxp + vy * dyp);
  t[LBM_T_E3 * plane + i] = vx * fxv + vy * fyv;
  t[LBM_T_E4 * plane + i] = -(sxx * dxux + sxy * dyux_n + sxy * dxuy_n + syy * dyuy);
  t[LBM_T_LHS_Z * plane + i] = (3.0 * ens[2] - 4.0 * ens[1] + ens[0]) / 2.0;
  t[LBM_T_Z2 * plane + i] = -ens[2] * (dxux + dyuy);
  t[LBM_T_USQ * plane + i] = vx * vx + vy * vy;
  double* ax = a.aux;
  ax[A_E * plane + i] = en[2];
  ax[A_OM2 * plane + i] = ens[2];
  ax[A_W * plane + i] = om[2];
  ax[A_SXX * plane + i] = sxx;
  ax[A_SYY * plane + i] = syy;
  ax[A_SXY * plane + i] = sxy;
}

__global__ void __launch_bounds__(256) k_bal_b(PassArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const int nx = a.nx, ny = a.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t i = static_cast<size_t>(y) * nx + x;
  const double* ux = a.ux[2];
  const double* uy = a.uy[2];
  const double* rho = a.rho[2];
  const double* ax = a.aux;
  const double* E = ax + A_E * plane;
  const double* Om = ax + A_OM2 * plane;
  const double* W = ax + A_W * plane;
  const double* sxx = ax + A_SXX * plane;
  const double* syy = ax + A_SYY * plane;
  const double* sxy = ax + A_SXY * plane;
  const bool forced = a.fx != nullptr;
  // x-derivatives: E u_x, u.sigma_x, Omega u_x, sigma_xx, sigma_xy, omega, F_y/rho
  // y-derivatives: E u_y, u.sigma_y, Omega u_y, sigma_xy, sigma_yy, omega, F_x/rho
  double dEx = 0, dEy = 0, dSx = 0, dSy = 0, dOx = 0, dOy = 0;
  double dxsxx = 0, dysxy = 0, dxsxy = 0, dysyy = 0, dxw = 0, dyw = 0, dxf = 0, dyf = 0;
#pragma unroll 1
  for (int m = 1; m <= 4; ++m) {
    const double c = kFd8[m - 1];
    const size_t xp = static_cast<size_t>(y) * nx + wrap_add(x, m, nx);
    const size_t xm = static_cast<size_t>(y) * nx + wrap_add(x, -m, nx);
    const size_t yp = static_cast<size_t>(wrap_add(y, m, ny)) * nx + x;
    const size_t ym = static_cast<size_t>(wrap_add(y, -m, ny)) * nx + x;
    {
      const double uxp = ux[xp], uxm = ux[xm], uyp = uy[xp], uym = uy[xm];
      const double sxxp = sxx[xp], sxxm = sxx[xm], sxyp = sxy[xp], sxym = sxy[xm];
      dEx += c * (E[xp] * uxp - E[xm] * uxm);
      dSx += c * ((uxp * sxxp + uyp * sxyp) - (uxm * sxxm + uym * sxym));
      dOx += c * (Om[xp] * uxp - Om[xm] * uxm);
      dxsxx += c * (sxxp - sxxm);
      dxsxy += c * (sxyp - sxym);
      dxw += c * (W[xp] - W[xm]);
      if (forced) dxf += c * (a.fy[xp] / rho[xp] - a.fy[xm] / rho[xm]);
    }
    {
      const double uxp = ux[yp], uxm = ux[ym], uyp = uy[yp], uym = uy[ym];
      const double sxyp = sxy[yp], sxym = sxy[ym], syyp = syy[yp], syym = syy[ym];
      dEy += c * (E[yp] * uyp - E[ym] * uym);
      dSy += c * ((uxp * sxyp + uyp * syyp) - (uxm * sxym + uym * syym));
      dOy += c * (Om[yp] * uyp - Om[ym] * uym);
      dysxy += c * (sxyp - sxym);
      dysyy += c * (syyp - syym);
      dyw += c * (W[yp] - W[ym]);
      if (forced) dyf += c * (a.fx[yp] / rho[yp] - a.fx[ym] / rho[ym]);
    }
  }
  const double r = rho[i];
  const double hx = (dxsxx + dysxy) / r;
  const double hy = (dxsxy + dysyy) / r;
  const double w = W[i];
  double* t = a.terms;
  t[LBM_T_E1 * plane + i] = -(dEx + dEy);
  t[LBM_T_E5 * plane + i] = dSx + dSy;
  t[LBM_T_Z1 * plane + i] = -(dOx + dOy);
  t[LBM_T_Z3 * plane + i] = forced ? w * (dxf - dyf) : 0.0;
  t[LBM_T_Z4 * plane + i] = hx * dyw - hy * dxw;
  a.aux[A_HX * plane + i] = hx;
  a.aux[A_HY * plane + i] = hy;
}

__global__ void __launch_bounds__(256) k_bal_c(PassArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const int nx = a.nx, ny = a.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t i = static_cast<size_t>(y) * nx + x;
  const double* W = a.aux + A_W * plane;
  const double* hx = a.aux + A_HX * plane;
  const double* hy = a.aux + A_HY * plane;
  a.terms[LBM_T_Z5 * plane + i] = fd8_x(F2{W, hy, nx}, x, y, nx) - fd8_y(F2{W, hx, nx}, x, y, ny);
}

// ---- the same passes on two sites per thread ----------------------------------------------
// Thread (x / 2, y) evaluates sites x and x + 1 (x even, nx even, every field
// 16-byte aligned) with 16-byte loads: a row segment x - 4 .. x + 5 serves both
// sites' x-differences, one pair per row their y-differences.  Each site's
// arithmetic is the one-site kernels' expression for expression, so the
// results are bitwise the same; the passes take about half as many vector
// memory instructions per site, which is what limits the one-site kernels.
__device__ __forceinline__ double2 ld2(const double* f, size_t row, int x) {
  return *reinterpret_cast<const double2*>(f + row + x);
}
__device__ __forceinline__ void st2(double* f, size_t i, double a, double b) {
  *reinterpret_cast<double2*>(f + i) = make_double2(a, b);
}
// the auxiliary fields are stored non-temporal: passes B and C read them back
// from HBM (eight fields of N^2 doubles do not stay in the caches)
__device__ __forceinline__ void st2nt(double* f, size_t i, double a, double b) {
  __builtin_nontemporal_store(a, f + i);
  __builtin_nontemporal_store(b, f + i + 1);
}
// values at columns x - 4 .. x + 5 of one row (x and nx even)
__device__ __forceinline__ void seg10(const double* f, size_t row, int x, int nx, double (&v)[10]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    int xx = x - 4 + 2 * q;
    xx += xx < 0 ? nx : 0;
    xx -= xx >= nx ? nx : 0;
    const double2 p = ld2(f, row, xx);
    v[2 * q] = p.x;
    v[2 * q + 1] = p.y;
  }
}
// Eq. 18 along x at the pair's two sites from a 10-value segment, accumulated
// offset by offset as in the one-site kernels
__device__ __forceinline__ void dx_pair(const double (&v)[10], double (&d)[2]) {
#pragma unroll
  for (int m = 1; m <= 4; ++m) {
    const double c = kFd8[m - 1];
    d[0] += c * (v[4 + m] - v[4 - m]);
    d[1] += c * (v[5 + m] - v[5 - m]);
  }
}

// Workgroup sums of the term fields a paired pass writes, for the field means
// of the tables: the 256 threads' values go through LDS, 32 threads per field add
// eight each and a 32-lane butterfly adds those, so the order is fixed.
// psum[field * blocks + block], block = blockIdx.y * gridDim.x + blockIdx.x.
// Table output of a paired pass, per term field F: the exclusive prefix sums of
// the raw values along the wave's 128 sites of row y (a wave is one row of the
// workgroup: lanes x / 2 - tile start), entries x and x + 1 of the field's table
// row y + 1 (entry c: the sum over the tile's sites before c), the last pair's
// inclusive sum also at entry nx (non-temporal stores: the column pass reads them
// back from HBM), and the 128-site total for the row carries.
// Sites past the grid's width count as zero.  The column pass later adds the
// carries from the tiles to the left and centres the values on the field's mean.
template <int... F>
__device__ __forceinline__ void row_scan_store(const PassArgs& a, const double (*o)[2], bool live, int x,
                                               int y) {
  constexpr int NF = sizeof...(F);
  constexpr int fld[NF] = {F...};
  const int lane = threadIdx.x;
  const size_t ld = static_cast<size_t>(a.ld);
  double* row = a.sat + static_cast<size_t>(y + 1) * NT * ld + x;
  const bool last = x + 2 == a.nx;
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const double o0 = live ? o[k][0] : 0.0;
    const double o1 = live ? o[k][1] : 0.0;
    double incl = o0 + o1;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double t = __shfl_up(incl, off, 64);
      incl += lane >= off ? t : 0.0;
    }
    double excl = __shfl_up(incl, 1, 64);
    excl = lane == 0 ? 0.0 : excl;
    if (live) {
      double* p = row + fld[k] * ld;
      __builtin_nontemporal_store(excl, p);
      __builtin_nontemporal_store(excl + o0, p + 1);
      if (last) __builtin_nontemporal_store(incl, p + 2);
    }
    if (lane == 63 && y < a.ny)
      a.rtot[(static_cast<size_t>(y) * NT + fld[k]) * gridDim.x + blockIdx.x] = incl;
  }
}

template <int... F>
__device__ __forceinline__ void block_field_sums(const double (&v)[sizeof...(F)], double* psum) {
  constexpr int NF = sizeof...(F);
  static_assert(NF * 32 <= 256, "32 threads per field");
  constexpr int fld[NF] = {F...};
  __shared__ double sh[NF][256];
  const int t = threadIdx.y * 64 + threadIdx.x;
#pragma unroll
  for (int f = 0; f < NF; ++f) sh[f][t] = v[f];
  __syncthreads();
  const int f = t >> 5, l = t & 31;
  double acc = 0.0;
  if (f < NF) {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += sh[f][l + 32 * j];
  }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 32);
  if (l == 0 && f < NF) {
    int field = fld[0];
#pragma unroll
    for (int k = 1; k < NF; ++k) field = f == k ? fld[k] : field;
    const size_t blocks = static_cast<size_t>(gridDim.x) * gridDim.y;
    psum[field * blocks + blockIdx.y * gridDim.x + blockIdx.x] = acc;
  }
}

__global__ void __launch_bounds__(256) k_bal_a2(PassArgs a) {
  const int nx = a.nx, ny = a.ny;
  // threads past the grid's edge evaluate the last pair of their row (or the
  // last row) and store nothing: every thread takes part in the workgroup sums
  const int xt = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
  const int yt = blockIdx.y * blockDim.y + threadIdx.y;
  const bool live = xt < nx && yt < ny;
  const int x = xt < nx ? xt : nx - 2;
  const int y = yt < ny ? yt : ny - 1;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t row = static_cast<size_t>(y) * nx;
  const size_t i = row + x;
  double dxuy[3][2] = {}, dyux[3][2] = {};
  double dxux[2] = {}, dyuy[2] = {}, dxr[2] = {}, dyr[2] = {};
  double cux[3][2], cuy[3][2], crho[3][2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double v[10];
    seg10(a.uy[k], row, x, nx, v);
    dx_pair(v, dxuy[k]);
    cuy[k][0] = v[4];
    cuy[k][1] = v[5];
  }
  {
    double v[10];
    seg10(a.ux[2], row, x, nx, v);
    dx_pair(v, dxux);
    cux[2][0] = v[4];
    cux[2][1] = v[5];
    seg10(a.rho[2], row, x, nx, v);
    dx_pair(v, dxr);
    crho[2][0] = v[4];
    crho[2][1] = v[5];
  }
#pragma unroll 1
  for (int m = 1; m <= 4; ++m) {
    const double c = kFd8[m - 1];
    const size_t rp = static_cast<size_t>(wrap_add(y, m, ny)) * nx;
    const size_t rm = static_cast<size_t>(wrap_add(y, -m, ny)) * nx;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double2 p = ld2(a.ux[k], rp, x), q = ld2(a.ux[k], rm, x);
      dyux[k][0] += c * (p.x - q.x);
      dyux[k][1] += c * (p.y - q.y);
    }
    {
      const double2 p = ld2(a.uy[2], rp, x), q = ld2(a.uy[2], rm, x);
      dyuy[0] += c * (p.x - q.x);
      dyuy[1] += c * (p.y - q.y);
    }
    {
      const double2 p = ld2(a.rho[2], rp, x), q = ld2(a.rho[2], rm, x);
      dyr[0] += c * (p.x - q.x);
      dyr[1] += c * (p.y - q.y);
    }
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double2 u = ld2(a.ux[k], row, x), r = ld2(a.rho[k], row, x);
    cux[k][0] = u.x;
    cux[k][1] = u.y;
    crho[k][0] = r.x;
    crho[k][1] = r.y;
  }
  double fxv[2] = {0.0, 0.0}, fyv[2] = {0.0, 0.0}, nuv[2] = {a.nu, a.nu};
  if (a.fx) {
    const double2 p = ld2(a.fx, row, x), q = ld2(a.fy, row, x);
    fxv[0] = p.x;
    fxv[1] = p.y;
    fyv[0] = q.x;
    fyv[1] = q.y;
  }
  if (a.nu_field) {
    const double2 p = ld2(a.nu_field, row, x);
    nuv[0] = p.x;
    nuv[1] = p.y;
  }
  double o[13][2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    double om[3], en[3], ens[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      om[k] = dxuy[k][s] - dyux[k][s];
      ens[k] = 0.5 * om[k] * om[k];
      const double vx = cux[k][s], vy = cuy[k][s];
      en[k] = 0.5 * crho[k][s] * (vx * vx + vy * vy);
    }
    const double dyux_n = dyux[2][s], dxuy_n = dxuy[2][s];
    const double r = crho[2][s], vx = cux[2][s], vy = cuy[2][s];
    const double dxp = dxr[s] / 3.0;
    const double dyp = dyr[s] / 3.0;
    const double nu = nuv[s];
    const double sxx = 2.0 * nu * r * dxux[s];
    const double syy = 2.0 * nu * r * dyuy[s];
    const double sxy = nu * r * (dxuy_n + dyux_n);
    o[0][s] = (3.0 * en[2] - 4.0 * en[1] + en[0]) / 2.0;
    o[1][s] = -(vx * dxp + vy * dyp);
    o[2][s] = vx * fxv[s] + vy * fyv[s];
    o[3][s] = -(sxx * dxux[s] + sxy * dyux_n + sxy * dxuy_n + syy * dyuy[s]);
    o[4][s] = (3.0 * ens[2] - 4.0 * ens[1] + ens[0]) / 2.0;
    o[5][s] = -ens[2] * (dxux[s] + dyuy[s]);
    o[6][s] = vx * vx + vy * vy;
    o[7][s] = en[2];
    o[8][s] = ens[2];
    o[9][s] = om[2];
    o[10][s] = sxx;
    o[11][s] = syy;
    o[12][s] = sxy;
  }
  if (live && a.terms) {
    double* t = a.terms;
    st2(t, LBM_T_LHS_E * plane + i, o[0][0], o[0][1]);
    st2(t, LBM_T_E2 * plane + i, o[1][0], o[1][1]);
    st2(t, LBM_T_E3 * plane + i, o[2][0], o[2][1]);
    st2(t, LBM_T_E4 * plane + i, o[3][0], o[3][1]);
    st2(t, LBM_T_LHS_Z * plane + i, o[4][0], o[4][1]);
    st2(t, LBM_T_Z2 * plane + i, o[5][0], o[5][1]);
    st2(t, LBM_T_USQ * plane + i, o[6][0], o[6][1]);
  }
  if (live) {
    double* ax = a.aux;
    if (!a.sat) {
      st2nt(ax, A_E * plane + i, o[7][0], o[7][1]);
      st2nt(ax, A_OM2 * plane + i, o[8][0], o[8][1]);
    }
    st2nt(ax, A_W * plane + i, o[9][0], o[9][1]);
    st2nt(ax, A_SXX * plane + i, o[10][0], o[10][1]);
    st2nt(ax, A_SYY * plane + i, o[11][0], o[11][1]);
    st2nt(ax, A_SXY * plane + i, o[12][0], o[12][1]);
  }
  if (a.sat) {
    row_scan_store<LBM_T_LHS_E, LBM_T_E2, LBM_T_E3, LBM_T_E4, LBM_T_LHS_Z, LBM_T_Z2, LBM_T_USQ>(a, o, live, x, yt);
  }
  double v[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) v[k] = live ? o[k][0] + o[k][1] : 0.0;
  block_field_sums<LBM_T_LHS_E, LBM_T_E2, LBM_T_E3, LBM_T_E4, LBM_T_LHS_Z, LBM_T_Z2, LBM_T_USQ>(v, a.psum);
}

__global__ void __launch_bounds__(256) k_bal_b2(PassArgs a) {
  const int nx = a.nx, ny = a.ny;
  // threads past the grid's edge evaluate the last pair of their row (or the
  // last row) and store nothing: every thread takes part in the workgroup sums
  const int xt = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
  const int yt = blockIdx.y * blockDim.y + threadIdx.y;
  const bool live = xt < nx && yt < ny;
  const int x = xt < nx ? xt : nx - 2;
  const int y = yt < ny ? yt : ny - 1;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t row = static_cast<size_t>(y) * nx;
  const size_t i = row + x;
  const double* ux = a.ux[2];
  const double* uy = a.uy[2];
  const double* rho = a.rho[2];
  const double* ax = a.aux;
  const double* W = ax + A_W * plane;
  const double* sxx = ax + A_SXX * plane;
  const double* syy = ax + A_SYY * plane;
  const double* sxy = ax + A_SXY * plane;
  const bool forced = a.fx != nullptr;
  // E = rho |u|^2 / 2 and Omega = omega^2 / 2 at the stencil points are formed
  // here from rho, u and omega (which the stencils load anyway), with pass A's
  // expressions, instead of being stored by pass A and read back
  auto energy = [](double r, double vx, double vy) { return 0.5 * r * (vx * vx + vy * vy); };
  auto enstrophy = [](double w) { return 0.5 * w * w; };
  double dEx[2] = {}, dEy[2] = {}, dSx[2] = {}, dSy[2] = {}, dOx[2] = {}, dOy[2] = {};
  double dxsxx[2] = {}, dysxy[2] = {}, dxsxy[2] = {}, dysyy[2] = {}, dxw[2] = {}, dyw[2] = {};
  double dxf[2] = {}, dyf[2] = {};
  double cw[2], cr[2];
  // y-derivatives first (fewer registers live across the x part), offset by
  // offset from pairs in rows y + m and y - m
#pragma unroll 1
  for (int m = 1; m <= 4; ++m) {
    const double c = kFd8[m - 1];
    const size_t rp = static_cast<size_t>(wrap_add(y, m, ny)) * nx;
    const size_t rm = static_cast<size_t>(wrap_add(y, -m, ny)) * nx;
    const double2 uxp = ld2(ux, rp, x), uxm = ld2(ux, rm, x), uyp = ld2(uy, rp, x), uym = ld2(uy, rm, x);
    const double2 sxyp = ld2(sxy, rp, x), sxym = ld2(sxy, rm, x), syyp = ld2(syy, rp, x), syym = ld2(syy, rm, x);
    const double2 rpp = ld2(rho, rp, x), rmm = ld2(rho, rm, x), Wp = ld2(W, rp, x), Wm = ld2(W, rm, x);
    const double pux[2] = {uxp.x, uxp.y}, mux[2] = {uxm.x, uxm.y}, puy[2] = {uyp.x, uyp.y}, muy[2] = {uym.x, uym.y};
    const double psxy[2] = {sxyp.x, sxyp.y}, msxy[2] = {sxym.x, sxym.y};
    const double psyy[2] = {syyp.x, syyp.y}, msyy[2] = {syym.x, syym.y};
    const double pr[2] = {rpp.x, rpp.y}, mr[2] = {rmm.x, rmm.y};
    const double pW[2] = {Wp.x, Wp.y}, mW[2] = {Wm.x, Wm.y};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const double pE = energy(pr[s], pux[s], puy[s]), mE = energy(mr[s], mux[s], muy[s]);
      const double pO = enstrophy(pW[s]), mO = enstrophy(mW[s]);
      dEy[s] += c * (pE * puy[s] - mE * muy[s]);
      dSy[s] += c * ((pux[s] * psxy[s] + puy[s] * psyy[s]) - (mux[s] * msxy[s] + muy[s] * msyy[s]));
      dOy[s] += c * (pO * puy[s] - mO * muy[s]);
      dysxy[s] += c * (psxy[s] - msxy[s]);
      dysyy[s] += c * (psyy[s] - msyy[s]);
      dyw[s] += c * (pW[s] - mW[s]);
    }
    if (forced) {
      const double2 fp = ld2(a.fx, rp, x), fm = ld2(a.fx, rm, x);
      const double pf[2] = {fp.x, fp.y}, mf[2] = {fm.x, fm.y};
#pragma unroll
      for (int s = 0; s < 2; ++s) dyf[s] += c * (pf[s] / pr[s] - mf[s] / mr[s]);
    }
  }
  // x-derivatives from 10-value row segments, a few fields at a time
  {
    double vux[10], vuy[10], vr[10];
    seg10(ux, row, x, nx, vux);
    seg10(uy, row, x, nx, vuy);
    seg10(rho, row, x, nx, vr);
    {
      double vsxx[10], vsxy[10];
      seg10(sxx, row, x, nx, vsxx);
      seg10(sxy, row, x, nx, vsxy);
#pragma unroll
      for (int m = 1; m <= 4; ++m) {
        const double c = kFd8[m - 1];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int p = 4 + s + m, q = 4 + s - m;
          dSx[s] += c * ((vux[p] * vsxx[p] + vuy[p] * vsxy[p]) - (vux[q] * vsxx[q] + vuy[q] * vsxy[q]));
          dxsxx[s] += c * (vsxx[p] - vsxx[q]);
          dxsxy[s] += c * (vsxy[p] - vsxy[q]);
        }
      }
    }
#pragma unroll
    for (int m = 1; m <= 4; ++m) {
      const double c = kFd8[m - 1];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int p = 4 + s + m, q = 4 + s - m;
        dEx[s] += c * (energy(vr[p], vux[p], vuy[p]) * vux[p] - energy(vr[q], vux[q], vuy[q]) * vux[q]);
      }
    }
    {
      double v[10];
      seg10(W, row, x, nx, v);
      dx_pair(v, dxw);
      cw[0] = v[4];
      cw[1] = v[5];
#pragma unroll
      for (int m = 1; m <= 4; ++m) {
        const double c = kFd8[m - 1];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int p = 4 + s + m, q = 4 + s - m;
          dOx[s] += c * (enstrophy(v[p]) * vux[p] - enstrophy(v[q]) * vux[q]);
        }
      }
    }
    if (forced) {
      double vf[10];
      seg10(a.fy, row, x, nx, vf);
#pragma unroll
      for (int m = 1; m <= 4; ++m) {
        const double c = kFd8[m - 1];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int p = 4 + s + m, q = 4 + s - m;
          dxf[s] += c * (vf[p] / vr[p] - vf[q] / vr[q]);
        }
      }
    }
    cr[0] = vr[4];
    cr[1] = vr[5];
  }
  double o[7][2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double r = cr[s];
    const double hx = (dxsxx[s] + dysxy[s]) / r;
    const double hy = (dxsxy[s] + dysyy[s]) / r;
    const double w = cw[s];
    o[0][s] = -(dEx[s] + dEy[s]);
    o[1][s] = dSx[s] + dSy[s];
    o[2][s] = -(dOx[s] + dOy[s]);
    o[3][s] = forced ? w * (dxf[s] - dyf[s]) : 0.0;
    o[4][s] = hx * dyw[s] - hy * dxw[s];
    o[5][s] = hx;
    o[6][s] = hy;
  }
  if (live && a.terms) {
    double* t = a.terms;
    st2(t, LBM_T_E1 * plane + i, o[0][0], o[0][1]);
    st2(t, LBM_T_E5 * plane + i, o[1][0], o[1][1]);
    st2(t, LBM_T_Z1 * plane + i, o[2][0], o[2][1]);
    st2(t, LBM_T_Z3 * plane + i, o[3][0], o[3][1]);
    st2(t, LBM_T_Z4 * plane + i, o[4][0], o[4][1]);
  }
  if (live) {
    st2nt(a.aux, A_HX * plane + i, o[5][0], o[5][1]);
    st2nt(a.aux, A_HY * plane + i, o[6][0], o[6][1]);
  }
  if (a.sat) {
    row_scan_store<LBM_T_E1, LBM_T_E5, LBM_T_Z1, LBM_T_Z3, LBM_T_Z4>(a, o, live, x, yt);
  }
  double v[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) v[k] = live ? o[k][0] + o[k][1] : 0.0;
  block_field_sums<LBM_T_E1, LBM_T_E5, LBM_T_Z1, LBM_T_Z3, LBM_T_Z4>(v, a.psum);
}

__global__ void __launch_bounds__(256) k_bal_c2(PassArgs a) {
  const int nx = a.nx, ny = a.ny;
  // threads past the grid's edge evaluate the last pair of their row (or the
  // last row) and store nothing: every thread takes part in the workgroup sums
  const int xt = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
  const int yt = blockIdx.y * blockDim.y + threadIdx.y;
  const bool live = xt < nx && yt < ny;
  const int x = xt < nx ? xt : nx - 2;
  const int y = yt < ny ? yt : ny - 1;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t row = static_cast<size_t>(y) * nx;
  const double* W = a.aux + A_W * plane;
  const double* hx = a.aux + A_HX * plane;
  const double* hy = a.aux + A_HY * plane;
  // Eq. 18 along x of W h_y and along y of W h_x, written as fd8_x / fd8_y
  double g[10];
  {
    double vw[10], vh[10];
    seg10(W, row, x, nx, vw);
    seg10(hy, row, x, nx, vh);
#pragma unroll
    for (int q = 0; q < 10; ++q) g[q] = vw[q] * vh[q];
  }
  double gy[2][9];  // rows y - 4 .. y + 4 of W h_x at the pair
#pragma unroll
  for (int m = -4; m <= 4; ++m) {
    if (m == 0) continue;
    const size_t r = static_cast<size_t>(wrap_add(y, m, ny)) * nx;
    const double2 w = ld2(W, r, x), h = ld2(hx, r, x);
    gy[0][m + 4] = w.x * h.x;
    gy[1][m + 4] = w.y * h.y;
  }
  double out[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double d1 = g[5 + s] - g[3 + s];
    const double d2 = g[6 + s] - g[2 + s];
    const double d3 = g[7 + s] - g[1 + s];
    const double d4 = g[8 + s] - g[0 + s];
    const double fx = (4.0 * d1 - d2 + (4.0 / 21.0) * d3 - (1.0 / 56.0) * d4) / 5.0;
    const double e1 = gy[s][5] - gy[s][3];
    const double e2 = gy[s][6] - gy[s][2];
    const double e3 = gy[s][7] - gy[s][1];
    const double e4 = gy[s][8] - gy[s][0];
    const double fy = (4.0 * e1 - e2 + (4.0 / 21.0) * e3 - (1.0 / 56.0) * e4) / 5.0;
    out[s] = fx - fy;
  }
  if (live && a.terms) st2(a.terms, LBM_T_Z5 * plane + row + x, out[0], out[1]);
  if (a.sat) {
    const double ot[1][2] = {{out[0], out[1]}};
    row_scan_store<LBM_T_Z5>(a, ot, live, x, yt);
  }
  const double v[1] = {live ? out[0] + out[1] : 0.0};
  block_field_sums<LBM_T_Z5>(v, a.psum);
}

// ---- field means ---------------------------------------------------------------------
constexpr int kRedThreads = 256;
constexpr int kMeanBlocks = 512;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// partials[field][block] = sum over the block's slice of field
__global__ void __launch_bounds__(kRedThreads) k_field_sums(const double* __restrict__ f, size_t n,
                                                             double* partials) {
  __shared__ double sh[kRedThreads / 64];
  const double* g = f + blockIdx.y * n;
  double acc = 0.0;
  for (size_t i = blockIdx.x * size_t(kRedThreads) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * kRedThreads)
    acc += g[i];
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) s += sh[w];
    partials[blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// means[f] = inv_n times the sum of partials[f][0 .. nblocks); each thread keeps
// eight loads in flight (eight running sums, added in a fixed order at the end)
__global__ void __launch_bounds__(kRedThreads) k_field_means(const double* __restrict__ partials,
                                                              int nblocks, double inv_n,
                                                              double* means) {
  __shared__ double sh[kRedThreads / 64];
  const double* p = partials + static_cast<size_t>(blockIdx.x) * nblocks;
  double a8[8] = {};
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += 8 * kRedThreads) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int b = b0 + q * kRedThreads;
      a8[q] += b < nblocks ? p[b] : 0.0;
    }
  }
  double acc = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) s += sh[w];
    means[blockIdx.x] = s * inv_n;
  }
}

// Table rows of one field are sat_ld(nx) doubles apart: nx + 1 rounded up to a
// multiple of 16, so every row starts on a 128-byte line (the workspace is
// 256-byte aligned) and the passes' 64-column segments (column passes, window
// walks) and 128-column segments (term passes) cover whole lines.
__host__ __device__ __forceinline__ int sat_ld(int nx) { return (nx + 16) & ~15; }

// ---- summed-area tables ------------------------------------------------------------------
// Row pass: P[f][y+1][x+1] = sum_{x' <= x} (g[f][y][x'] - mean_f); P[f][0][*] = P[f][*][0] = 0.
// One workgroup per (row, field); the row is consumed in coalesced segments of
// 256 values, each scanned across the workgroup (wavefront shuffles, then the
// four wavefront totals through LDS) and offset by the running total.
__global__ void __launch_bounds__(256) k_sat_rows(const double* __restrict__ g,
                                                  const double* __restrict__ means, double* sat,
                                                  int nx, int ny, int nf) {
  __shared__ double wsum[4];
  const int y = blockIdx.x;
  const int f = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t s = static_cast<size_t>(sat_ld(nx));
  const double mean = means[f];
  const double* row = g + f * plane + static_cast<size_t>(y) * nx;
  double* out = sat + (static_cast<size_t>(y + 1) * nf + f) * s;
  double carry = 0.0;
  for (int x0 = 0; x0 < nx; x0 += 256) {
    const int x = x0 + threadIdx.x;
    double v = x < nx ? row[x] - mean : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double t = __shfl_up(v, off, 64);
      if (lane >= off) v += t;
    }
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    double before = 0.0;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    const double total = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    if (x < nx) out[x + 1] = carry + (before + v);
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 0.0;
  if (y == 0) {
    double* top = sat + f * s;
    for (int xx = threadIdx.x; xx <= nx; xx += 256) top[xx] = 0.0;
  }
}

// Column pass: a workgroup of 64 columns x kColG row groups walks the table
// down in chunks of kColG x kColR rows.  Each thread holds its kColR rows of one
// column in registers; the group totals go through LDS, and each thread writes
// its rows back as running sums offset by the column's carry from the chunks
// above and by the totals of the groups above it in the chunk.  The table is
// read once and written once, both non-temporal (the table is far larger than the
// caches).  Every load is issued (at a clamped row and column) and its value
// selected away where it lies outside the table; an empty asm statement takes
// each loaded value, so the compiler cannot sink the loads into conditional
// blocks (one load in flight at a time) and a chunk's loads are all in flight
// together.  All workgroups of a 4096^2 table are resident at once.
//
// With CARRY, the rows hold the paired term passes' 128-site scans of the raw
// values instead (entry c the sum over its tile's sites before c; entry nx the
// last tile's total) and rcarry[(y * nf + f) * ntx + t] the centred sum of row y
// over the tiles left of tile t; each value is completed to the centred row
// prefix as it is loaded, entry + carry - mean x (sites summed in the tile).  A
// wave's 64 columns lie in one tile, so its carries are wave-uniform (scalar
// loads).  The pass also writes the zero top row.
constexpr int kColG = 4;
constexpr int kColR = 16;
constexpr int kScanTile = 128;  // sites of a row in one paired-pass wave
template <bool CARRY>
__global__ void __launch_bounds__(64 * kColG) k_sat_cols(double* sat, int nx, int ny, int nf,
                                                         const double* __restrict__ rcarry,
                                                         const double* __restrict__ means, int ntx) {
  __shared__ double sh[kColG][64];
  const int c = blockIdx.x * 64 + threadIdx.x;
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int f = blockIdx.y;
  double* P = sat + f * static_cast<size_t>(sat_ld(nx));
  const size_t s = static_cast<size_t>(sat_ld(nx)) * nf;  // between rows of one field
  const bool active = c <= nx;
  const int cl = active ? c : nx;
  // completion of the scanned rows: the wave's tile and the sites summed at this column
  const int tile = min(static_cast<int>(blockIdx.x) / (kScanTile / 64), ntx - 1);
  const double msum = CARRY ? means[f] * double(c - tile * kScanTile) : 0.0;
  const double* rc = CARRY ? rcarry + static_cast<size_t>(f) * ntx + tile : nullptr;
  const size_t rcs = static_cast<size_t>(nf) * ntx;  // between rows of the carries
  if (CARRY && g == 0 && active) P[c] = 0.0;  // top row
  double carry = 0.0;  // this column's sum over the rows above the chunk
  for (int y0 = 1; y0 <= ny; y0 += kColG * kColR) {
    const int ya = y0 + g * kColR;
    double v[kColR], k[kColR];
    double acc = 0.0;
    if constexpr (CARRY) {
#pragma unroll
      for (int q = 0; q < kColR; ++q) k[q] = rc[static_cast<size_t>((ya + q <= ny ? ya + q : ny) - 1) * rcs];
    }
#pragma unroll
    for (int q = 0; q < kColR; ++q) {
      const int yl = ya + q <= ny ? ya + q : ny;
      v[q] = __builtin_nontemporal_load(P + yl * s + cl);
    }
#pragma unroll
    for (int q = 0; q < kColR; ++q) {
      if constexpr (CARRY) asm volatile("" ::"s"(k[q]));
      asm volatile("" ::"v"(v[q]));
    }
#pragma unroll
    for (int q = 0; q < kColR; ++q) {
      const int y = ya + q;
      double t = v[q];
      if constexpr (CARRY) t = (t + k[q]) - msum;
      v[q] = (active && y <= ny) ? t : 0.0;
      acc += v[q];
    }
    sh[g][threadIdx.x] = acc;
    __syncthreads();
    double off = carry, tot = carry;
    for (int k = 0; k < kColG; ++k) {
      const double t = sh[k][threadIdx.x];
      if (k < g) off += t;
      tot += t;
    }
    __syncthreads();  // sh is rewritten by the next chunk
    if (active) {
      double run = off;
#pragma unroll
      for (int q = 0; q < kColR; ++q) {
        const int y = ya + q;
        run += v[q];
        if (y <= ny) __builtin_nontemporal_store(run, P + y * s + c);
      }
    }
    carry = tot;
  }
}

// ---- windows -----------------------------------------------------------------------------------
struct SatView {
  const double* P;  // [ny+1][nf][ld], entries x = 0 .. nx of each row used
  const double* means;
  int nx, ny;
  int nf;           // fields per table row
  int ld;           // sat_ld(nx): doubles between consecutive fields' rows
  // Q(y, x) for 0 <= y < 2 ny, 0 <= x < 2 nx: the periodic continuation of the
  // prefix table through its totals.
  __device__ __forceinline__ double Q(int f, int y, int x) const {
    const size_t s = static_cast<size_t>(ld) * nf;  // between rows of one field
    const double* p = P + f * static_cast<size_t>(ld);
    const int qy = y > ny ? 1 : 0;
    const int qx = x > nx ? 1 : 0;
    const int ym = y - qy * ny;
    const int xm = x - qx * nx;
    double v = p[ym * s + xm];
    if (qy) v += p[static_cast<size_t>(ny) * s + xm];
    if (qx) v += p[ym * s + nx];
    if (qy && qx) v += p[static_cast<size_t>(ny) * s + nx];
    return v;
  }
  __device__ __forceinline__ double box_mean(int f, int x0, int y0, int L) const {
    const double s = Q(f, y0 + L, x0 + L) - Q(f, y0, x0 + L) - Q(f, y0 + L, x0) + Q(f, y0, x0);
    return means[f] + s / (double(L) * double(L));
  }
};

__device__ void window_errors(const double (&m)[NT], double& dE, double& dZ, double& ma) {
  const double rE = (((m[LBM_T_E1] + m[LBM_T_E2]) + m[LBM_T_E3]) + m[LBM_T_E4]) + m[LBM_T_E5];
  const double denE = fmax(fmax(fmax(fabs(m[LBM_T_E1]), fabs(m[LBM_T_E2])),
                                fmax(fabs(m[LBM_T_E3]), fabs(m[LBM_T_E4]))),
                           fabs(m[LBM_T_E5]));
  const double rZ = (((m[LBM_T_Z1] + m[LBM_T_Z2]) + m[LBM_T_Z3]) + m[LBM_T_Z4]) + m[LBM_T_Z5];
  const double denZ = fmax(fmax(fmax(fabs(m[LBM_T_Z1]), fabs(m[LBM_T_Z2])),
                                fmax(fabs(m[LBM_T_Z3]), fabs(m[LBM_T_Z4]))),
                           fabs(m[LBM_T_Z5]));
  dE = denE > 0.0 ? fabs(rE - m[LBM_T_LHS_E]) / denE : __builtin_nan("");
  dZ = denZ > 0.0 ? fabs(rZ - m[LBM_T_LHS_Z]) / denZ : __builtin_nan("");
  ma = sqrt(m[LBM_T_USQ]) * 1.7320508075688772;  // / c_s, c_s = 1/sqrt(3)
}

// Running statistics: n, mean, M2, min, max, nan count.
// ---- histograms ---------------------------------------------------------------------------
// Bin of a finite value: the number of edges <= v (0 .. n).
__device__ __forceinline__ int hist_bin(const double* e, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (e[mid] <= v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// A workgroup's histogram of one quantity in LDS, flushed to the device counts
// with integer atomics (exact: the totals do not depend on the order).
struct LdsHist {
  unsigned* bins;
  const double* e;
  int n;
  __device__ __forceinline__ void add(double v) const {
    if (isfinite(v)) atomicAdd(&bins[hist_bin(e, n, v)], 1u);
  }
};
__device__ void lds_hist_init(unsigned* bins, double* e_lds, const double* e, int n) {
  for (int i = threadIdx.x; i <= n; i += blockDim.x) bins[i] = 0u;
  for (int i = threadIdx.x; i < n; i += blockDim.x) e_lds[i] = e[i];
}
__device__ void lds_hist_flush(const unsigned* bins, int n, unsigned long long* g) {
  for (int i = threadIdx.x; i <= n; i += blockDim.x)
    if (bins[i]) atomicAdd(&g[i], static_cast<unsigned long long>(bins[i]));
}

struct RS {
  double n, mean, m2, mn, mx, nan;
  __device__ void init() {
    n = mean = m2 = nan = 0.0;
    mn = 1e300;
    mx = -1e300;
  }
  __device__ void add(double v) {
    if (!isfinite(v)) {
      nan += 1.0;
      return;
    }
    n += 1.0;
    const double d = v - mean;
    mean += d / n;
    m2 += d * (v - mean);
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  __device__ void merge(const RS& b) {
    const double nn = n + b.n;
    if (b.n > 0.0) {
      const double d = b.mean - mean;
      mean = nn > 0.0 ? mean + d * (b.n / nn) : 0.0;
      m2 = m2 + b.m2 + d * d * (n * b.n / nn);
      n = nn;
      mn = fmin(mn, b.mn);
      mx = fmax(mx, b.mx);
    }
    nan += b.nan;
  }
};
constexpr int kRS = 6;
constexpr int kStatVals = 3 * kRS;  // dE, dZ, Ma

__device__ void rs_shfl_merge(RS& r, int off) {
  RS o;
  o.n = __shfl_xor(r.n, off, 64);
  o.mean = __shfl_xor(r.mean, off, 64);
  o.m2 = __shfl_xor(r.m2, off, 64);
  o.mn = __shfl_xor(r.mn, off, 64);
  o.mx = __shfl_xor(r.mx, off, 64);
  o.nan = __shfl_xor(r.nan, off, 64);
  // merge in a lane-independent order so every lane of a pair ends equal
  if ((threadIdx.x & off) == 0) {
    r.merge(o);
  } else {
    o.merge(r);
    r = o;
  }
}

__device__ void block_stats(RS (&r)[3], double* out) {
  __shared__ double sh[4][3][kRS];
  for (int q = 0; q < 3; ++q)
    for (int off = 1; off < 64; off <<= 1) rs_shfl_merge(r[q], off);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int q = 0; q < 3; ++q) {
      sh[wv][q][0] = r[q].n;
      sh[wv][q][1] = r[q].mean;
      sh[wv][q][2] = r[q].m2;
      sh[wv][q][3] = r[q].mn;
      sh[wv][q][4] = r[q].mx;
      sh[wv][q][5] = r[q].nan;
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / 64;
    for (int q = 0; q < 3; ++q) {
      RS acc;
      acc.init();
      for (int w = 0; w < nw; ++w) {
        RS b{sh[w][q][0], sh[w][q][1], sh[w][q][2], sh[w][q][3], sh[w][q][4], sh[w][q][5]};
        acc.merge(b);
      }
      out[q * kRS + 0] = acc.n;
      out[q * kRS + 1] = acc.mean;
      out[q * kRS + 2] = acc.m2;
      out[q * kRS + 3] = acc.mn;
      out[q * kRS + 4] = acc.mx;
      out[q * kRS + 5] = acc.nan;
    }
  }
}

constexpr int kWinThreads = 256;
constexpr int kWinMaxBlocks = 1024;

// Windows of side L at every corner (xy == nullptr: corner i = (i % nx, i / nx),
// i < count) or at the corners xy[i] (taken modulo the grid); optional maps
// (enumerated corners only) and histograms of the three quantities.
template <bool HIST>
__global__ void __launch_bounds__(kWinThreads) k_windows(SatView v, int L, const int32_t* __restrict__ xy,
                                                         size_t count, double* maps, double* partials,
                                                         const double* __restrict__ edges, int nedges,
                                                         unsigned long long* hist) {
  RS r[3];
  for (int q = 0; q < 3; ++q) r[q].init();
  LdsHist hh[3] = {};
  if constexpr (HIST) {
    __shared__ unsigned bins[3][LBM_MAX_EDGES + 1];
    __shared__ double e[3][LBM_MAX_EDGES];
    for (int q = 0; q < 3; ++q) {
      lds_hist_init(bins[q], e[q], edges + q * nedges, nedges);
      hh[q] = LdsHist{bins[q], e[q], nedges};
    }
    __syncthreads();
  }
  const size_t plane = static_cast<size_t>(v.nx) * v.ny;
  for (size_t i = blockIdx.x * size_t(kWinThreads) + threadIdx.x; i < count;
       i += size_t(gridDim.x) * kWinThreads) {
    int x0, y0;
    if (xy) {
      x0 = xy[2 * i] % v.nx;
      y0 = xy[2 * i + 1] % v.ny;
      x0 += x0 < 0 ? v.nx : 0;
      y0 += y0 < 0 ? v.ny : 0;
    } else {
      x0 = static_cast<int>(i % v.nx);
      y0 = static_cast<int>(i / v.nx);
    }
    double m[NT];
#pragma unroll
    for (int f = 0; f < NT; ++f) m[f] = v.box_mean(f, x0, y0, L);
    double dE, dZ, ma;
    window_errors(m, dE, dZ, ma);
    r[0].add(dE);
    r[1].add(dZ);
    r[2].add(ma);
    if constexpr (HIST) {
      hh[0].add(dE);
      hh[1].add(dZ);
      hh[2].add(ma);
    }
    if (maps && !xy) {
      maps[i] = dE;
      maps[plane + i] = dZ;
      maps[2 * plane + i] = ma;
    }
  }
  if constexpr (HIST) {
    __syncthreads();
    for (int q = 0; q < 3; ++q) lds_hist_flush(hh[q].bins, nedges, hist + q * (nedges + 1));
  }
  block_stats(r, partials + blockIdx.x * kStatVals);
}

__global__ void __launch_bounds__(kWinThreads) k_stats_final(const double* __restrict__ partials,
                                                             int nblocks, double* out) {
  RS r[3];
  for (int q = 0; q < 3; ++q) r[q].init();
  for (int b = threadIdx.x; b < nblocks; b += kWinThreads)
    for (int q = 0; q < 3; ++q) {
      const double* p = partials + b * kStatVals + q * kRS;
      RS o{p[0], p[1], p[2], p[3], p[4], p[5]};
      r[q].merge(o);
    }
  block_stats(r, out);
}

// Pool slot i = (size, quantity): the statistics of this call, or merged with
// the slot's earlier contents (Chan's pairwise update).
__global__ void k_stats_pool(const double* __restrict__ cur, double* pool, int nslots, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots) return;
  const double* c = cur + static_cast<size_t>(i) * kRS;
  double* p = pool + static_cast<size_t>(i) * kRS;
  RS a{c[0], c[1], c[2], c[3], c[4], c[5]};
  if (accumulate) {
    RS b{p[0], p[1], p[2], p[3], p[4], p[5]};
    b.merge(a);
    a = b;
  }
  p[0] = a.n;
  p[1] = a.mean;
  p[2] = a.m2;
  p[3] = a.mn;
  p[4] = a.mx;
  p[5] = a.nan;
}

__global__ void k_zero_u64(unsigned long long* p, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0ull;
}

constexpr int kSumVals = 3 * 6;

struct SumStat {
  double n, s1, s2, mn, mx, nan;
  __device__ void init() {
    n = s1 = s2 = nan = 0.0;
    mn = 1e300;
    mx = -1e300;
  }
  // add(v) when c (wave-uniform in the walks) holds, else nothing.  Both adds
  // are without branches (a lane-divergent branch costs exec-mask bookkeeping
  // and register copies on every window) and give the same values as skipping
  // v when it is not finite.
  __device__ __forceinline__ void add_if(double v, bool c) {
    const bool fin = isfinite(v);
    const bool ok = c && fin;
    const double w = ok ? v : 0.0;
    n += ok ? 1.0 : 0.0;
    nan += (c && !fin) ? 1.0 : 0.0;
    s1 += w;
    s2 += w * w;
    mn = ok ? fmin(mn, v) : mn;
    mx = ok ? fmax(mx, v) : mx;
  }
  // Keeps the running values in registers at this point of the program: in a
  // fully unrolled walk the compiler would otherwise defer every window's update
  // to the end and hold all the window values live meanwhile.
  __device__ __forceinline__ void pin() {
    asm volatile("" : "+v"(n), "+v"(s1), "+v"(s2), "+v"(mn), "+v"(mx), "+v"(nan));
  }
  __device__ __forceinline__ void add(double v) {
    const bool ok = isfinite(v);
    const double w = ok ? v : 0.0;
    n += ok ? 1.0 : 0.0;
    nan += ok ? 0.0 : 1.0;
    s1 += w;
    s2 += w * w;
    mn = ok ? fmin(mn, v) : mn;
    mx = ok ? fmax(mx, v) : mx;
  }
};

__device__ void sum_stats_block(SumStat (&r)[3], double* out) {
  __shared__ double sh[4][kSumVals];
  double v[kSumVals];
  for (int q = 0; q < 3; ++q) {
    v[q * 6 + 0] = r[q].n;
    v[q * 6 + 1] = r[q].s1;
    v[q * 6 + 2] = r[q].s2;
    v[q * 6 + 3] = r[q].mn;
    v[q * 6 + 4] = r[q].mx;
    v[q * 6 + 5] = r[q].nan;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < kSumVals; ++k) {
      const double o = __shfl_xor(v[k], off, 64);
      const int kind = k % 6;
      v[k] = kind == 3 ? fmin(v[k], o) : (kind == 4 ? fmax(v[k], o) : v[k] + o);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < kSumVals; ++k) sh[wv][k] = v[k];
  __syncthreads();
  if (threadIdx.x < kSumVals) {
    const int k = threadIdx.x, kind = k % 6;
    double a = sh[0][k];
    for (int w = 1; w < 4; ++w) {
      const double o = sh[w][k];
      a = kind == 3 ? fmin(a, o) : (kind == 4 ? fmax(a, o) : a + o);
    }
    out[k] = a;
  }
  __syncthreads();
}

// The same partial slot from a workgroup whose windows all belong to field group
// grp: only that group's six values are reduced (the same butterfly and fixed
// order), the other groups' slots get the empty statistics.  A walk then keeps
// one SumStat per side in registers instead of three.
__device__ void sum_stats_group(const SumStat& r, int grp, double* out) {
  __shared__ double sh[4][6];
  double v[6] = {r.n, r.s1, r.s2, r.mn, r.mx, r.nan};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double o = __shfl_xor(v[k], off, 64);
      v[k] = k == 3 ? fmin(v[k], o) : (k == 4 ? fmax(v[k], o) : v[k] + o);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < 6; ++k) sh[wv][k] = v[k];
  __syncthreads();
  if (threadIdx.x < kSumVals) {
    const int k = threadIdx.x % 6, q = threadIdx.x / 6;
    double a = k == 3 ? 1e300 : (k == 4 ? -1e300 : 0.0);
    if (q == grp) {
      a = sh[0][k];
      for (int w = 1; w < 4; ++w) {
        const double o = sh[w][k];
        a = k == 3 ? fmin(a, o) : (k == 4 ? fmax(a, o) : a + o);
      }
    }
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

// Work split of the windows of one box side L (see k_windows_strided): strips
// of 256 columns, residues j < L, and segments of at most kStrideSteps corner
// rows of each residue's sequence.
constexpr int kStrideSteps = 16;
struct StrideGrid {
  int strips, G, S;
  long long blocks;  // per field group
};
StrideGrid stride_grid(int nx, int ny, int L) {
  StrideGrid g;
  g.strips = (nx + 255) / 256;
  const int Q = (ny + L - 1) / L;
  g.G = (Q + kStrideSteps - 1) / kStrideSteps;
  g.S = (Q + g.G - 1) / g.G;
  g.blocks = static_cast<long long>(g.strips) * L * g.G;
  return g;
}

// Fields [F0, F0 + NF) of the windows of one workgroup: group 0 (LHS_E and
// the five energy terms) gives delta^E, group 1 (LHS_Omega and the five
// enstrophy terms) delta^Omega, group 2 (|u|^2) the Mach number, each into
// its own statistics slot.
// The window's statistic from its box means: Ma_V (one field, |u|^2) or the
// balancing error |sum of the five terms - LHS| / largest |term| (six fields),
// as window_errors.
template <int NF>
__device__ __forceinline__ double window_value(const double (&m)[NF]) {
  if constexpr (NF == 1) {
    return sqrt(m[0]) * 1.7320508075688772;  // Ma_V = sqrt(<|u|^2>) / c_s, c_s = 1/sqrt(3)
  } else {
    const double rs = (((m[1] + m[2]) + m[3]) + m[4]) + m[5];
    const double den = fmax(fmax(fmax(fabs(m[1]), fabs(m[2])), fmax(fabs(m[3]), fabs(m[4]))), fabs(m[5]));
    return den > 0.0 ? fabs(rs - m[0]) / den : __builtin_nan("");
  }
}

template <int F0, int NF>
__device__ __forceinline__ void stride_windows(const SatView& v, int L, int x0, int y0, int S,
                                               double* maps, SumStat& r, const LdsHist* h) {
  const int nx = v.nx, ny = v.ny;
  const unsigned s = static_cast<unsigned>(v.ld) * v.nf;  // between rows of one field
  const unsigned fs = static_cast<unsigned>(v.ld);        // between fields of one row
  const double inv = 1.0 / (double(L) * double(L));
  const bool qx = x0 + L > nx;
  const unsigned xm = qx ? x0 + L - nx : x0 + L;
  const double* P = v.P + F0 * fs;
  // uniform over the workgroup: some window of the strip wraps in x, some
  // window of the sequence wraps in y
  const bool any_qx = (x0 - static_cast<int>(threadIdx.x)) + 255 + L > nx;
  const bool any_qy = y0 + S * L > ny;
  // the table's last row (column totals) at the window's columns, for rows
  // continued past y = ny
  double t0[NF], t1[NF], tn[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) t0[k] = t1[k] = tn[k] = 0.0;
  if (any_qy) {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      t0[k] = P[k * fs + ny * s + x0];
      t1[k] = P[k * fs + ny * s + xm];
      tn[k] = P[k * fs + ny * s + nx];
    }
  }
  // Q(y, x0 + L) - Q(y, x0) for table row y in [0, 2 ny), continued
  // periodically through the row and column totals, in two parts: the raw
  // loads of a row, and the differences.  The next row's loads are issued
  // before the current window is evaluated, so they are in flight during its
  // arithmetic.
  struct Raw {
    double b0[NF], b1[NF], bn[NF];
  };
  auto load = [&](int y, Raw& w) {
    const unsigned ym = y > ny ? y - ny : y;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const double* p = P + k * fs;
      w.b0[k] = p[ym * s + x0];
      w.b1[k] = p[ym * s + xm];
      w.bn[k] = any_qx ? p[ym * s + nx] : 0.0;
    }
  };
  auto finish = [&](int y, const Raw& w, double (&d)[NF]) {
    const bool qy = y > ny;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      double c0 = w.b0[k];
      double c1 = qx ? w.b1[k] + w.bn[k] : w.b1[k];
      if (qy) {
        c0 += t0[k];
        c1 += t1[k];
        c1 = qx ? c1 + tn[k] : c1;
      }
      d[k] = c1 - c0;
    }
  };
  // the field means in registers (a load inside the loop would sit behind the
  // next row's loads and wait for them)
  double mu[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) mu[k] = v.means[F0 + k];
  double dt[NF];  // per field, the difference across the current window's top row
  Raw rn;
  load(y0, rn);
  finish(y0, rn, dt);
  if (S > 0 && y0 < ny) load(y0 + L, rn);
  for (int i = 0; i < S && y0 < ny; ++i, y0 += L) {
    double db[NF], m[NF];
    finish(y0 + L, rn, db);
    if (i + 1 < S && y0 + L < ny) load(y0 + 2 * L, rn);
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      m[k] = mu[k] + (db[k] - dt[k]) * inv;
      dt[k] = db[k];  // the bottom row is the next window's top row
    }
    const double val = window_value<NF>(m);
    r.add(val);
    if (h) h->add(val);
    if (maps) maps[static_cast<unsigned>(y0) * nx + x0] = val;
  }
}

// One box side L per launch.  Workgroup (group, strip, j, g) takes one field
// group and the window corners x0 in its 256-column strip and
// y0 = j + L q, q = g S .. g S + S - 1: along that sequence the bottom row of a
// window is the top row of the next, so each table row is loaded once per side
// (plus one row per segment) and reused from registers.  Workgroups are
// numbered so that neighbouring strips share an XCD (and its L2, which serves
// the columns x0 + L past the strip), and the three field groups alternate
// (logical index = 3 x block + group): each XCD's contiguous range holds equal
// shares of the six-field groups and of the one-field group, so no XCD runs
// out of work while another still walks its six-field windows.
template <bool HIST>
__global__ void __launch_bounds__(256) k_windows_strided(SatView v, int L, int strips, int S, int nblocks,
                                                         int per_xcd, double* maps, double* partials,
                                                         const double* __restrict__ edges, int nedges,
                                                         unsigned long long* hist) {
  const int b = blockIdx.x;
  const int logical = (b & 7) * per_xcd + (b >> 3);
  if (logical >= 3 * nblocks) return;  // uniform over the workgroup
  const int grp = logical % 3;
  const int wb = logical / 3;
  const int strip = wb % strips;
  const int rest = wb / strips;
  const int j = rest % L, g = rest / L;
  const int x0 = strip * 256 + threadIdx.x;
  const int y0 = j + L * (g * S);
  const size_t plane = static_cast<size_t>(v.nx) * v.ny;
  SumStat r;
  r.init();
  LdsHist hh{nullptr, nullptr, 0};
  if constexpr (HIST) {
    __shared__ unsigned bins[LBM_MAX_EDGES + 1];
    __shared__ double e[LBM_MAX_EDGES];
    lds_hist_init(bins, e, edges + grp * nedges, nedges);
    hh = LdsHist{bins, e, nedges};
    __syncthreads();
  }
  const LdsHist* h = HIST ? &hh : nullptr;
  if (x0 < v.nx && y0 < v.ny) {
    if (grp == 0)
      stride_windows<LBM_T_LHS_E, 6>(v, L, x0, y0, S, maps, r, h);
    else if (grp == 1)
      stride_windows<LBM_T_LHS_Z, 6>(v, L, x0, y0, S, maps ? maps + plane : nullptr, r, h);
    else
      stride_windows<LBM_T_USQ, 1>(v, L, x0, y0, S, maps ? maps + 2 * plane : nullptr, r, h);
  }
  if constexpr (HIST) {
    __syncthreads();
    lds_hist_flush(hh.bins, nedges, hist + grp * (nedges + 1));
  }
  sum_stats_group(r, grp, partials + static_cast<size_t>(logical) * kSumVals);
}

// Sides L and 2 L at the same corners in one walk (no histograms, no maps):
// along the sequence y0, y0 + L, ... a row's raw values at x0, x0 + L and
// x0 + 2 L give both sides' differences; the side-L window whose top is row
// j - 1 and the side-2L window whose top is row j - 2 both end at row j.
// The table rows are read once for the two sides.
template <int F0, int NF>
__device__ __forceinline__ void stride_windows2(const SatView& v, int L, int x0, int y0, int S,
                                                SumStat& r1, SumStat& r2) {
  const int nx = v.nx, ny = v.ny;
  const unsigned s = static_cast<unsigned>(v.ld) * v.nf;
  const unsigned fs = static_cast<unsigned>(v.ld);
  const int L2 = 2 * L;
  const double inv1 = 1.0 / (double(L) * double(L));
  const double inv2 = 1.0 / (double(L2) * double(L2));
  const bool qx1 = x0 + L > nx, qx2 = x0 + L2 > nx;
  const unsigned xm1 = qx1 ? x0 + L - nx : x0 + L;
  const unsigned xm2 = qx2 ? x0 + L2 - nx : x0 + L2;
  const double* P = v.P + F0 * fs;
  const int nwin = min(S, (ny - y0 + L - 1) / L);  // corners y0 + w L < ny, w < S
  const bool any_qx = (x0 - static_cast<int>(threadIdx.x)) + 255 + L2 > nx;
  const bool any_qy = y0 + (nwin + 1) * L > ny;
  double t0[NF], t1[NF], t2[NF], tn[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) t0[k] = t1[k] = t2[k] = tn[k] = 0.0;
  if (any_qy) {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const double* p = P + k * fs + ny * s;
      t0[k] = p[x0];
      t1[k] = p[xm1];
      t2[k] = p[xm2];
      tn[k] = p[nx];
    }
  }
  struct Raw {
    double b0[NF], b1[NF], b2[NF], bn[NF];
  };
  auto load = [&](int y, Raw& w) {
    const unsigned ym = y > ny ? y - ny : y;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const double* p = P + k * fs + ym * s;
      w.b0[k] = p[x0];
      w.b1[k] = p[xm1];
      w.b2[k] = p[xm2];
      w.bn[k] = any_qx ? p[nx] : 0.0;
    }
  };
  // the same operations as the one-side walk, for each side
  auto finish = [&](int y, const Raw& w, double (&d1)[NF], double (&d2)[NF]) {
    const bool qy = y > ny;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      double c0 = w.b0[k];
      double c1 = qx1 ? w.b1[k] + w.bn[k] : w.b1[k];
      double c2 = qx2 ? w.b2[k] + w.bn[k] : w.b2[k];
      if (qy) {
        c0 += t0[k];
        c1 += t1[k];
        c1 = qx1 ? c1 + tn[k] : c1;
        c2 += t2[k];
        c2 = qx2 ? c2 + tn[k] : c2;
      }
      d1[k] = c1 - c0;
      d2[k] = c2 - c0;
    }
  };
  double mu[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) mu[k] = v.means[F0 + k];
  double a1[NF];          // side L: difference of the row above (top of window j - 1)
  double a2[NF], b2[NF];  // side 2 L: differences of rows j - 2 and j - 1
  Raw rn;
  load(y0, rn);
  finish(y0, rn, a1, b2);
  load(y0 + L, rn);
  for (int j = 1; j <= nwin + 1; ++j) {
    const int y = y0 + j * L;
    double d1[NF], d2[NF];
    finish(y, rn, d1, d2);
    if (j <= nwin) load(y + L, rn);
    if (j - 1 < nwin) {
      double m[NF];
#pragma unroll
      for (int k = 0; k < NF; ++k) m[k] = mu[k] + (d1[k] - a1[k]) * inv1;
      r1.add(window_value<NF>(m));
    }
    if (j >= 2) {
      double m[NF];
#pragma unroll
      for (int k = 0; k < NF; ++k) m[k] = mu[k] + (d2[k] - a2[k]) * inv2;
      r2.add(window_value<NF>(m));
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      a1[k] = d1[k];
      a2[k] = b2[k];
      b2[k] = d2[k];
    }
  }
}

// Buffer resource over `bytes` bytes from a wave-uniform address (raw buffer,
// 32-bit elements format word of the gfx9 family).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), 0x00020000);
}
__device__ __forceinline__ double buf_load_f64(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(voff),
                                                                         static_cast<int>(soff), 0));
}

// stride_windows2 for a workgroup whose windows neither wrap in x (every lane's
// x0 + 2 L <= nx) nor in y (the sequence's last row y0 + (nwin + 1) L <= ny):
// no totals rows or columns, no selects.  A table row's fields are read through a
// buffer resource built per row from its wave-uniform address (scalar
// registers), with each lane's byte offsets x0, x0 + L, x0 + 2 L fixed for the
// walk and the field offsets as scalar offsets, so no address arithmetic runs on
// the vector units.  The raw loads of rows j + 1 and j + 2 are in flight while
// row j's windows are evaluated (two buffers by the parity of j, and the
// differences of the two previous rows kept by parity as well).  The walk is
// unrolled completely (nwin <= kStrideSteps): loads past the sequence's last row
// re-read that row and the windows that do not exist are masked out, so there
// are no branches and every value keeps its registers.  The window values are
// computed exactly as in stride_windows2.
template <int F0, int NF>
__device__ __forceinline__ void stride_windows2_inner(const SatView& v, int L, int x0, int y0, int nwin,
                                                      SumStat& r1, SumStat& r2) {
  const unsigned fsb = static_cast<unsigned>(v.ld) * 8u;  // bytes between fields of one row
  const double* base = v.P + static_cast<size_t>(F0) * v.ld;
  const size_t rs = static_cast<size_t>(v.ld) * v.nf;     // doubles between table rows
  const unsigned o0 = static_cast<unsigned>(x0) * 8u;
  const unsigned o1 = static_cast<unsigned>(x0 + L) * 8u;
  const unsigned o2 = static_cast<unsigned>(x0 + 2 * L) * 8u;
  const double inv1 = 1.0 / (double(L) * double(L));
  const double inv2 = 1.0 / (double(2 * L) * double(2 * L));
  double mu[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) mu[k] = v.means[F0 + k];
  struct Raw {
    double b0[NF], b1[NF], b2[NF];
  };
  const int last = nwin + 1;  // rows 0 .. last of the sequence are read
  auto load = [&](int j, Raw& w) {
    const int y = y0 + min(j, last) * L;
    __amdgpu_buffer_rsrc_t r = raw_rsrc(base + static_cast<size_t>(y) * rs, NF * fsb);
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      w.b0[k] = buf_load_f64(r, o0, k * fsb);
      w.b1[k] = buf_load_f64(r, o1, k * fsb);
      w.b2[k] = buf_load_f64(r, o2, k * fsb);
    }
  };
  Raw rw[2];
  double h1[2][NF], h2[2][NF];  // differences of the rows j - 1, j - 2 by parity
  load(0, rw[0]);
  load(1, rw[1]);
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    h1[0][k] = rw[0].b1[k] - rw[0].b0[k];
    h2[0][k] = rw[0].b2[k] - rw[0].b0[k];
  }
  load(2, rw[0]);
  auto row_step = [&](auto parity, int j) {
    constexpr int P = decltype(parity)::value;
    double d1[NF], d2[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      d1[k] = rw[P].b1[k] - rw[P].b0[k];
      d2[k] = rw[P].b2[k] - rw[P].b0[k];
    }
    load(j + 2, rw[P]);
    double m1[NF], m2[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      m1[k] = mu[k] + (d1[k] - h1[P ^ 1][k]) * inv1;
      m2[k] = mu[k] + (d2[k] - h2[P][k]) * inv2;
    }
    r1.add_if(window_value<NF>(m1), j - 1 < nwin);
    r2.add_if(window_value<NF>(m2), j >= 2 && j <= last);
    r1.pin();
    r2.pin();
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      h1[P][k] = d1[k];
      h2[P][k] = d2[k];
    }
  };
#pragma unroll
  for (int jj = 0; jj < (kStrideSteps + 2) / 2; ++jj) {
    row_step(std::integral_constant<int, 1>{}, 2 * jj + 1);
    row_step(std::integral_constant<int, 0>{}, 2 * jj + 2);
  }
}

// Sides L and 2 L per launch, the work split of k_windows_strided for side L;
// the partials of side 2 L follow those of side L.
struct PairWork {
  int grp, strip, y0, x0, nwin;
  int slot;  // partial slot, 3 x work item + group
  bool live;
};
template <int G0, int NG>
__device__ __forceinline__ PairWork pair_work(const SatView& v, int L, int strips, int S, int nblocks,
                                              int per_xcd) {
  const int b = blockIdx.x;
  const int logical = (b & 7) * per_xcd + (b >> 3);
  PairWork w{};
  w.live = logical < NG * nblocks;
  if (!w.live) return w;
  w.grp = G0 + logical % NG;  // groups alternate, as in k_windows_strided
  const int wb = logical / NG;
  w.slot = 3 * wb + w.grp;
  w.strip = wb % strips;
  const int rest = wb / strips;
  const int j = rest % L, g = rest / L;
  w.x0 = w.strip * 256 + threadIdx.x;
  w.y0 = j + L * (g * S);
  w.nwin = min(S, (v.ny - w.y0 + L - 1) / L);
  return w;
}

// Whether a pair-walk workgroup's windows stay inside the table (no lane's
// windows wrap in x, its sequence does not wrap in y): uniform over the workgroup.
__device__ __forceinline__ bool pair_inner(const SatView& v, int L, const PairWork& w) {
  return w.strip * 256 + 255 + 2 * L <= v.nx && w.y0 + (w.nwin + 1) * L <= v.ny && w.y0 < v.ny;
}

// Groups G0 .. G0 + NG - 1 of the pair walk: the six-field groups (0, 1) in one
// launch and the one-field group (2) in another, so that each is compiled for its
// own register count (the one-field walk runs at higher occupancy).
template <int G0, int NG>
__global__ void __launch_bounds__(256) k_windows_pair(SatView v, int L, int strips, int S, int nblocks,
                                                      int per_xcd, double* partials) {
  const PairWork w = pair_work<G0, NG>(v, L, strips, S, nblocks, per_xcd);
  if (!w.live) return;  // uniform over the workgroup
  SumStat r1, r2;
  r1.init();
  r2.init();
  if (pair_inner(v, L, w)) {
    if (G0 == 2)
      stride_windows2_inner<LBM_T_USQ, 1>(v, L, w.x0, w.y0, w.nwin, r1, r2);
    else if (w.grp == 0)
      stride_windows2_inner<LBM_T_LHS_E, 6>(v, L, w.x0, w.y0, w.nwin, r1, r2);
    else
      stride_windows2_inner<LBM_T_LHS_Z, 6>(v, L, w.x0, w.y0, w.nwin, r1, r2);
  } else if (w.x0 < v.nx && w.y0 < v.ny) {
    if (G0 == 2)
      stride_windows2<LBM_T_USQ, 1>(v, L, w.x0, w.y0, S, r1, r2);
    else if (w.grp == 0)
      stride_windows2<LBM_T_LHS_E, 6>(v, L, w.x0, w.y0, S, r1, r2);
    else
      stride_windows2<LBM_T_LHS_Z, 6>(v, L, w.x0, w.y0, S, r1, r2);
  }
  sum_stats_group(r1, w.grp, partials + static_cast<size_t>(w.slot) * kSumVals);
  sum_stats_group(r2, w.grp, partials + (static_cast<size_t>(3) * nblocks + w.slot) * kSumVals);
}

// The window walks' partials are merged in two stages.  First stage: set
// blockIdx.y of partial blocks (nblocks blocks of kSumVals values each, sets
// one after the other) is cut into kStatMid contiguous chunks; workgroup g
// reads chunk g with 252 threads as 14 rows x 18 values, so that consecutive
// threads read consecutive doubles, and combines its rows in a fixed order
// into mid[set][g].
constexpr int kStatMid = 64;
constexpr int kStatRows = 256 / kSumVals;
__global__ void __launch_bounds__(256) k_sum_stats_mid(const double* __restrict__ partials, int nblocks,
                                                       double* __restrict__ mid) {
  __shared__ double sh[kStatRows][kSumVals];
  const int t = threadIdx.x;
  const int row = t / kSumVals, j = t - row * kSumVals;
  const int kind = j % 6;
  const double* p = partials + static_cast<size_t>(blockIdx.y) * nblocks * kSumVals;
  const int per = (nblocks + kStatMid - 1) / kStatMid;
  const int b0 = blockIdx.x * per;
  const int b1 = min(nblocks, b0 + per);
  double acc = kind == 3 ? 1e300 : (kind == 4 ? -1e300 : 0.0);
  if (row < kStatRows) {
    for (int b = b0 + row; b < b1; b += kStatRows) {
      const double v = p[static_cast<size_t>(b) * kSumVals + j];
      acc = kind == 3 ? fmin(acc, v) : (kind == 4 ? fmax(acc, v) : acc + v);
    }
    sh[row][j] = acc;
  }
  __syncthreads();
  if (t < kSumVals) {
    double r = sh[0][t];
    for (int q = 1; q < kStatRows; ++q) {
      const double v = sh[q][t];
      r = kind == 3 ? fmin(r, v) : (kind == 4 ? fmax(r, v) : r + v);
    }
    mid[(static_cast<size_t>(blockIdx.y) * kStatMid + blockIdx.x) * kSumVals + t] = r;
  }
}

// Second stage: workgroup q combines mid[q] and writes the three statistics in
// the (n, mean, M2, min, max, nan) layout of the Welford path to out_q.
__global__ void __launch_bounds__(256) k_sum_stats_final(const double* __restrict__ mid, double* out0,
                                                         double* out1) {
  SumStat r[3];
  for (int q = 0; q < 3; ++q) r[q].init();
  const double* part = mid + static_cast<size_t>(blockIdx.x) * kStatMid * kSumVals;
  for (int b = threadIdx.x; b < kStatMid; b += 256)
    for (int q = 0; q < 3; ++q) {
      const double* p = part + static_cast<size_t>(b) * kSumVals + q * 6;
      r[q].n += p[0];
      r[q].s1 += p[1];
      r[q].s2 += p[2];
      r[q].mn = fmin(r[q].mn, p[3]);
      r[q].mx = fmax(r[q].mx, p[4]);
      r[q].nan += p[5];
    }
  __shared__ double fin[kSumVals];
  sum_stats_block(r, fin);
  double* out = blockIdx.x == 0 ? out0 : out1;
  if (threadIdx.x < 3) {
    const int q = threadIdx.x;
    const double n = fin[q * 6 + 0];
    const double mean = n > 0.0 ? fin[q * 6 + 1] / n : 0.0;
    const double m2 = n > 0.0 ? fmax(fin[q * 6 + 2] - n * mean * mean, 0.0) : 0.0;
    out[q * kRS + 0] = n;
    out[q * kRS + 1] = mean;
    out[q * kRS + 2] = m2;
    out[q * kRS + 3] = fin[q * 6 + 3];
    out[q * kRS + 4] = fin[q * 6 + 4];
    out[q * kRS + 5] = fin[q * 6 + 5];
  }
}

// Per explicit window: the NT box means, then delta^E, delta^Omega and Ma_V.
__global__ void k_window_terms(SatView v, const int32_t* __restrict__ win, int nwin, double* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nwin) return;
  const int x0 = win[3 * k], y0 = win[3 * k + 1], L = win[3 * k + 2];
  double m[NT];
  for (int f = 0; f < NT; ++f) {
    m[f] = v.box_mean(f, x0, y0, L);
    out[k * LBM_NWVALS + f] = m[f];
  }
  double dE, dZ, ma;
  window_errors(m, dE, dZ, ma);
  out[k * LBM_NWVALS + LBM_W_DE] = dE;
  out[k * LBM_NWVALS + LBM_W_DZ] = dZ;
  out[k * LBM_NWVALS + LBM_W_MA] = ma;
}

int stat_blocks(size_t count) {
  size_t b = (count + kWinThreads - 1) / kWinThreads;
  if (b > kWinMaxBlocks) b = kWinMaxBlocks;
  return static_cast<int>(b < 1 ? 1 : b);
}

}  // namespace

int balance_grid_ok(int nx, int ny) {
  const unsigned long long elems = static_cast<unsigned long long>(NT) * static_cast<unsigned long long>(sat_ld(nx)) *
                                   (static_cast<unsigned long long>(ny) + 1);
  if (elems >= (1ull << 32))
    return fail(LBM_E_UNSUPPORTED,
                "balance of a %d x %d grid: its prefix tables hold %llu elements, beyond the 2^32 "
                "the window walks address",
                nx, ny, elems);
  return LBM_OK;
}

size_t balance_ws_bytes(int nx, int ny) {
  Carver c(nullptr, 0);
  carve_balance(c, nx, ny);
  return c.used + 256;
}

BalanceWs carve_balance(Carver& c, int nx, int ny) {
  const size_t plane = static_cast<size_t>(nx) * ny;
  const size_t splane = static_cast<size_t>(sat_ld(nx)) * (ny + 1);
  BalanceWs w;
  w.terms = c.take<double>(NT * plane);
  w.aux = c.take<double>(NAUX * plane);
  w.sat = c.take<double>(NT * splane);
  w.rtot = c.take<double>(static_cast<size_t>(NT) * ny * ((nx / 2 + 63) / 64));
  w.means = c.take<double>(16);
  size_t np = static_cast<size_t>(kWinMaxBlocks) * kStatVals;
  for (int L = 1; L <= (nx < ny ? nx : ny); ++L) {
    // sides paired with 2 L keep both sides' partials
    const size_t sides = 2 * L <= (nx < ny ? nx : ny) ? 2 : 1;
    const size_t need = sides * 3 * static_cast<size_t>(stride_grid(nx, ny, L).blocks) * kSumVals;
    if (np < need) np = need;
  }
  // after them, the field-sum partials: the paired term passes' workgroup sums
  // or the fallback reduction's block sums
  const size_t pass_blocks = static_cast<size_t>((nx / 2 + 63) / 64) * ((ny + 3) / 4);
  w.partials = c.take<double>(np + static_cast<size_t>(NT) * std::max<size_t>(kMeanBlocks, pass_blocks));
  w.partials_cap = np;
  w.stats = c.take<double>(static_cast<size_t>(kMaxSizes) * kStatVals);
  w.sstats = c.take<double>(static_cast<size_t>(kMaxSizes) * kStatVals);
  w.pool = c.take<double>(2 * static_cast<size_t>(kMaxSizes) * kStatVals);
  w.edges = c.take<double>(3 * static_cast<size_t>(LBM_MAX_EDGES));
  w.hist = c.take<unsigned long long>(2 * static_cast<size_t>(kMaxSizes) * 3 * (LBM_MAX_EDGES + 1));
  w.wterms = c.take<double>(static_cast<size_t>(kMaxWindows) * LBM_NWVALS);
  w.windows = c.take<int32_t>(static_cast<size_t>(kMaxWindows) * 3);
  return w;
}

int balance_terms(const lbm_balance_input& in, const BalanceWs& ws) {
  return balance_terms(in, ws, true, nullptr);
}

int balance_terms(const lbm_balance_input& in, const BalanceWs& ws, bool planes, bool* table) {
  hipStream_t s = static_cast<hipStream_t>(in.stream);
  const int nx = in.nx, ny = in.ny;
  PassArgs a;
  for (int k = 0; k < 3; ++k) {
    a.rho[k] = in.rho[k];
    a.ux[k] = in.ux[k];
    a.uy[k] = in.uy[k];
  }
  a.fx = in.fx;
  a.fy = in.fy;
  a.nu = in.nu;
  a.nu_field = in.nu_field;
  a.nx = nx;
  a.ny = ny;
  a.terms = ws.terms;
  a.aux = ws.aux;
  a.sat = nullptr;
  a.rtot = nullptr;
  a.ld = sat_ld(nx);
  // two sites per thread where the grid width is even and every field is
  // 16-byte aligned (bitwise the same results), else one site per thread
  auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  bool paired = nx % 2 == 0 && al16(a.terms) && al16(a.aux) && al16(a.fx) && al16(a.fy) &&
                al16(a.nu_field);
  for (int k = 0; k < 3; ++k) paired = paired && al16(a.rho[k]) && al16(a.ux[k]) && al16(a.uy[k]);
  a.psum = ws.partials + ws.partials_cap;
  dim3 blk(64, 4);
  if (table) *table = paired;
  if (paired) {
    if (table) {
      // the passes scan their rows into the prefix table; the planes only on request
      a.sat = ws.sat;
      a.rtot = ws.rtot;
      if (!planes) a.terms = nullptr;
    }
    dim3 grd((nx / 2 + 63) / 64, (ny + 3) / 4);
    hipLaunchKernelGGL(k_bal_a2, grd, blk, 0, s, a);
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_bal_b2, grd, blk, 0, s, a);
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_bal_c2, grd, blk, 0, s, a);
    LBM_HIP(hipGetLastError());
    // the field means from the passes' workgroup sums
    hipLaunchKernelGGL(k_field_means, dim3(NT), dim3(kRedThreads), 0, s, a.psum,
                       static_cast<int>(grd.x * grd.y), 1.0 / (double(nx) * ny), ws.means);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
  }
  dim3 grd((nx + 63) / 64, (ny + 3) / 4);
  hipLaunchKernelGGL(k_bal_a, grd, blk, 0, s, a);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bal_b, grd, blk, 0, s, a);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bal_c, grd, blk, 0, s, a);
  LBM_HIP(hipGetLastError());
  return field_means(ws.terms, NT, nx, ny, a.psum, ws.means, s);
}

int field_means(const double* g, int nf, int nx, int ny, double* partials, double* means,
                hipStream_t s) {
  const size_t plane = static_cast<size_t>(nx) * ny;
  int mb = static_cast<int>((plane + kRedThreads - 1) / kRedThreads);
  if (mb > kMeanBlocks) mb = kMeanBlocks;
  hipLaunchKernelGGL(k_field_sums, dim3(mb, nf), dim3(kRedThreads), 0, s, g, plane, partials);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_field_means, dim3(nf), dim3(kRedThreads), 0, s, partials, mb,
                     1.0 / double(plane), means);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

int sat_build(const double* g, int nf, const double* means, double* sat, int nx, int ny,
              hipStream_t s) {
  hipLaunchKernelGGL(k_sat_rows, dim3(ny, nf), dim3(256), 0, s, g, means, sat, nx, ny, nf);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sat_cols<false>, dim3((nx + 1 + 63) / 64, nf), dim3(64, kColG), 0, s, sat, nx, ny, nf,
                     static_cast<const double*>(nullptr), static_cast<const double*>(nullptr), 0);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

namespace {
// Row carries of the scanned table rows, in place: thread (y, f) turns the
// 128-site totals of row y into their centred exclusive prefix sums,
// carry(t) = sum over t' < t of (total(t') - mean_f x sites of tile t').
__global__ void __launch_bounds__(256) k_row_carries(double* rtot, const double* __restrict__ means, int nx,
                                                     int ny, int ntx) {
  const int i = blockIdx.x * 256 + threadIdx.x;  // y * 13 + f
  if (i >= ny * NT) return;
  const double m = means[i % NT];
  double* r = rtot + static_cast<size_t>(i) * ntx;
  double run = 0.0;
  for (int t = 0; t < ntx; ++t) {
    const double tot = r[t];
    r[t] = run;
    const int w = nx - t * kScanTile < kScanTile ? nx - t * kScanTile : kScanTile;
    run += tot - m * double(w);
  }
}
}  // namespace

int balance_table(const lbm_balance_input& in, const BalanceWs& ws, bool planes) {
  hipStream_t s = static_cast<hipStream_t>(in.stream);
  const int nx = in.nx, ny = in.ny;
  bool paired = false;
  if (int rc = balance_terms(in, ws, planes, &paired)) return rc;
  if (!paired) return sat_build(ws.terms, NT, ws.means, ws.sat, nx, ny, s);
  const int ntx = (nx / 2 + 63) / 64;
  hipLaunchKernelGGL(k_row_carries, dim3((ny * NT + 255) / 256), dim3(256), 0, s, ws.rtot,
                     static_cast<const double*>(ws.means), nx, ny, ntx);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sat_cols<true>, dim3((nx + 1 + 63) / 64, NT), dim3(64, kColG), 0, s, ws.sat, nx, ny, NT,
                     static_cast<const double*>(ws.rtot), static_cast<const double*>(ws.means), ntx);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

namespace {
// out[y][x] = scale * (sum of field f over the L x L periodic box whose lower
// corner is (y + off, x + off)), from its mean-centred table.
__global__ void __launch_bounds__(256) k_box_map(SatView v, int f, int L, int off, double scale,
                                                 double* out) {
  const size_t plane = static_cast<size_t>(v.nx) * v.ny;
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < plane; i += size_t(gridDim.x) * 256) {
    int x0 = static_cast<int>(i % v.nx) + off;
    int y0 = static_cast<int>(i / v.nx) + off;
    x0 += x0 < 0 ? v.nx : 0;
    y0 += y0 < 0 ? v.ny : 0;
    const double box = v.Q(f, y0 + L, x0 + L) - v.Q(f, y0, x0 + L) - v.Q(f, y0 + L, x0) + v.Q(f, y0, x0);
    out[i] = scale * (box + v.means[f] * double(L) * double(L));
  }
}
}  // namespace

int box_map(const double* sat, const double* means, int nf, int f, int L, int off, double scale,
            double* out, int nx, int ny, hipStream_t s) {
  SatView v{sat, means, nx, ny, nf, sat_ld(nx)};
  const size_t plane = static_cast<size_t>(nx) * ny;
  int g = static_cast<int>((plane + 255) / 256);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_box_map, dim3(g), dim3(256), 0, s, v, f, L, off, scale, out);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

namespace {
void fill_stats(const double* q, int L, lbm_balance_stats& o) {
  o = lbm_balance_stats{};
  o.L = L;
  auto fill = [](const double* r, int64_t& cnt, int64_t* nan, double& mean, double& sd, double& mn,
                 double& mx) {
    cnt = static_cast<int64_t>(r[0]);
    if (nan) *nan = static_cast<int64_t>(r[5]);
    if (cnt > 0) {
      mean = r[1];
      sd = std::sqrt(r[2] / r[0]);
      mn = r[3];
      mx = r[4];
    } else {
      mean = sd = mn = mx = NAN;
    }
  };
  fill(q + 0 * kRS, o.count_dE, &o.nan_dE, o.mean_dE, o.std_dE, o.min_dE, o.max_dE);
  fill(q + 1 * kRS, o.count_dZ, &o.nan_dZ, o.mean_dZ, o.std_dZ, o.min_dZ, o.max_dZ);
  fill(q + 2 * kRS, o.count_Ma, nullptr, o.mean_Ma, o.std_Ma, o.min_Ma, o.max_Ma);
}

int launch_windows(bool hist, const SatView& v, int L, const int32_t* xy, size_t count, int blocks,
                   double* maps, double* partials, const double* edges, int nedges,
                   unsigned long long* h, hipStream_t s) {
  if (hist)
    hipLaunchKernelGGL(k_windows<true>, dim3(blocks), dim3(kWinThreads), 0, s, v, L, xy, count, maps, partials,
                       edges, nedges, h);
  else
    hipLaunchKernelGGL(k_windows<false>, dim3(blocks), dim3(kWinThreads), 0, s, v, L, xy, count, maps,
                       partials, edges, nedges, h);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}
}  // namespace

int validate_balance_extra(int nsizes, const lbm_balance_stats* out, const lbm_balance_extra* x) {
  if (!x) return LBM_OK;
  if (x->accumulate != 0 && x->accumulate != 1) return fail(LBM_E_INVALID, "accumulate must be 0 or 1");
  if (x->edges) {
    if (x->nedges < 1 || x->nedges > LBM_MAX_EDGES)
      return fail(LBM_E_INVALID, "nedges must be in [1, %d]", LBM_MAX_EDGES);
    for (int q = 0; q < 3; ++q)
      for (int i = 0; i < x->nedges; ++i) {
        const double e = x->edges[q * x->nedges + i];
        if (!std::isfinite(e)) return fail(LBM_E_INVALID, "histogram edge %d of quantity %d not finite", i, q);
        if (i > 0 && !(e > x->edges[q * x->nedges + i - 1]))
          return fail(LBM_E_INVALID, "histogram edges of quantity %d not strictly increasing", q);
      }
  } else if (x->hist || x->sample_hist) {
    return fail(LBM_E_INVALID, "histograms need edges");
  }
  if (x->hist && !out) return fail(LBM_E_INVALID, "hist needs the all-corner statistics (out)");
  if (x->sample_counts) {
    if (!x->sample_out) return fail(LBM_E_INVALID, "sample_counts needs sample_out");
    long long tot = 0;
    for (int k = 0; k < nsizes; ++k) {
      if (x->sample_counts[k] < 0) return fail(LBM_E_INVALID, "sample count %d is negative", k);
      tot += x->sample_counts[k];
    }
    if (tot > 0x7fffffffLL) return fail(LBM_E_INVALID, "too many sampled windows");
    if (tot > 0 && !x->sample_xy) return fail(LBM_E_INVALID, "sample_xy is NULL");
  } else if (x->sample_out || x->sample_hist || x->sample_xy) {
    return fail(LBM_E_INVALID, "sampled windows need sample_counts");
  }
  return LBM_OK;
}

namespace {

// Merge of nsets sets of nblocks window-walk partials (ws.partials, one set
// after the other) into out0 (and out1), through the first-stage sums kept
// after the window partials.
int merge_sum_stats(const BalanceWs& ws, int nblocks, int nsets, double* out0, double* out1, hipStream_t s) {
  double* mid = ws.partials + ws.partials_cap;
  hipLaunchKernelGGL(k_sum_stats_mid, dim3(kStatMid, nsets), dim3(256), 0, s, ws.partials, nblocks, mid);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_stats_final, dim3(nsets), dim3(256), 0, s, mid, out0, out1);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

// Statistics over every corner for each box side: window kernels, the merge of
// their partials into ws.stats, then the pool (started anew unless acc).
int corner_stats(const SatView& v, const BalanceWs& ws, const int32_t* sizes, int nsizes, double* dmaps,
                 bool hist, int ne, unsigned long long* hall, size_t hslot, int acc, hipStream_t s) {
  const int nx = v.nx, ny = v.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  // Without histograms or maps, a side L whose double 2 L is also asked for (and
  // is not the whole domain) shares one walk of the tables with it.
  int twin[kMaxSizes];  // index of side 2 L, or -2 for a side done with its half
  for (int k = 0; k < nsizes; ++k) twin[k] = -1;
  if (!hist && !dmaps) {
    for (int k = 0; k < nsizes; ++k) {
      if (twin[k] != -1) continue;
      const int L = sizes[k];
      if (2 * L > (nx < ny ? nx : ny) || (2 * L == nx && 2 * L == ny)) continue;
      for (int k2 = 0; k2 < nsizes; ++k2)
        if (k2 != k && twin[k2] == -1 && sizes[k2] == 2 * L) {
          twin[k] = k2;
          twin[k2] = -2;
          break;
        }
    }
  }
  for (int k = 0; k < nsizes; ++k) {
    const int L = sizes[k];
    if (twin[k] == -2) continue;
    if (twin[k] >= 0) {
      const StrideGrid g = stride_grid(nx, ny, L);
      if (2 * 3 * g.blocks * kSumVals > static_cast<long long>(ws.partials_cap))
        return fail(LBM_E_INVALID, "box sides %d, %d: window partials exceed the workspace", L, 2 * L);
      const int nb = static_cast<int>(g.blocks);
      const int per_xcd6 = (2 * nb + 7) / 8, per_xcd1 = (nb + 7) / 8;
      hipLaunchKernelGGL((k_windows_pair<0, 2>), dim3(per_xcd6 * 8), dim3(256), 0, s, v, L, g.strips, g.S, nb,
                         per_xcd6, ws.partials);
      LBM_HIP(hipGetLastError());
      hipLaunchKernelGGL((k_windows_pair<2, 1>), dim3(per_xcd1 * 8), dim3(256), 0, s, v, L, g.strips, g.S, nb,
                         per_xcd1, ws.partials);
      LBM_HIP(hipGetLastError());
      if (int rc = merge_sum_stats(ws, 3 * nb, 2, ws.stats + static_cast<size_t>(k) * kStatVals,
                                   ws.stats + static_cast<size_t>(twin[k]) * kStatVals, s))
        return rc;
      continue;
    }
    double* maps = dmaps ? dmaps + static_cast<size_t>(k) * 3 * plane : nullptr;
    unsigned long long* hk = hall + static_cast<size_t>(k) * hslot;
    if (L == nx && L == ny) {
      if (int rc = launch_windows(hist, v, L, nullptr, 1, 1, maps, ws.partials, ws.edges, ne, hk, s))
        return rc;
      hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kWinThreads), 0, s, ws.partials, 1,
                         ws.stats + static_cast<size_t>(k) * kStatVals);
      LBM_HIP(hipGetLastError());
      continue;
    }
    const StrideGrid g = stride_grid(nx, ny, L);
    if (3 * g.blocks * kSumVals > static_cast<long long>(ws.partials_cap))
      return fail(LBM_E_INVALID, "box side %d: window partials exceed the workspace", L);
    const int nb = static_cast<int>(g.blocks);
    const int per_xcd = (3 * nb + 7) / 8;
    if (hist)
      hipLaunchKernelGGL(k_windows_strided<true>, dim3(per_xcd * 8), dim3(256), 0, s, v, L, g.strips, g.S,
                         nb, per_xcd, maps, ws.partials, ws.edges, ne, hk);
    else
      hipLaunchKernelGGL(k_windows_strided<false>, dim3(per_xcd * 8), dim3(256), 0, s, v, L, g.strips, g.S,
                         nb, per_xcd, maps, ws.partials, ws.edges, ne, hk);
    LBM_HIP(hipGetLastError());
    if (int rc = merge_sum_stats(ws, 3 * nb, 1, ws.stats + static_cast<size_t>(k) * kStatVals, nullptr, s))
      return rc;
  }
  if (nsizes > 0) {
    hipLaunchKernelGGL(k_stats_pool, dim3((3 * nsizes + 63) / 64), dim3(64), 0, s, ws.stats, ws.pool,
                       3 * nsizes, acc);
    LBM_HIP(hipGetLastError());
  }
  return LBM_OK;
}

}  // namespace

namespace {

// Per-workgroup sums of omega^2 / 2, omega = d_x u_y - d_y u_x by Eq. 18.
__global__ void __launch_bounds__(kRedThreads) k_enstrophy(const double* __restrict__ ux,
                                                            const double* __restrict__ uy, int nx, int ny,
                                                            double* partials) {
  __shared__ double sh[kRedThreads / 64];
  const size_t plane = static_cast<size_t>(nx) * ny;
  const fd8::F1 gx{ux, nx}, gy{uy, nx};
  double acc = 0.0;
  for (size_t i = blockIdx.x * size_t(kRedThreads) + threadIdx.x; i < plane; i += size_t(gridDim.x) * kRedThreads) {
    const int x = static_cast<int>(i % nx), y = static_cast<int>(i / nx);
    const double w = fd8::fd8_x(gy, x, y, nx) - fd8::fd8_y(gx, x, y, ny);
    acc += 0.5 * w * w;
  }
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) s += sh[w];
    partials[blockIdx.x] = s;
  }
}

}  // namespace

int global_enstrophy(const double* ux, const double* uy, int nx, int ny, double* partials, int max_blocks,
                     double* dev_out, double* host_out, hipStream_t s) {
  const size_t plane = static_cast<size_t>(nx) * ny;
  const int nb = static_cast<int>(std::max<size_t>(1, std::min<size_t>(max_blocks, (plane + kRedThreads - 1) / kRedThreads)));
  hipLaunchKernelGGL(k_enstrophy, dim3(nb), dim3(kRedThreads), 0, s, ux, uy, nx, ny, partials);
  LBM_HIP(hipGetLastError());
  // one fixed-order sum of the partials (the field-mean kernel with weight 1)
  hipLaunchKernelGGL(k_field_means, dim3(1), dim3(kRedThreads), 0, s, partials, nb, 1.0, dev_out);
  LBM_HIP(hipGetLastError());
  LBM_HIP(hipMemcpyAsync(host_out, dev_out, sizeof(double), hipMemcpyDeviceToHost, s));
  LBM_HIP(hipStreamSynchronize(s));
  return LBM_OK;
}

int run_balance_async(const lbm_balance_input& in, const BalanceWs& ws, const int32_t* sizes, int nsizes,
                      double* host_stats) {
  hipStream_t s = static_cast<hipStream_t>(in.stream);
  if (int rc = balance_table(in, ws, false)) return rc;
  SatView v{ws.sat, ws.means, in.nx, in.ny, NT, sat_ld(in.nx)};
  if (int rc = corner_stats(v, ws, sizes, nsizes, nullptr, false, 0, ws.hist, 0, 0, s)) return rc;
  LBM_HIP(hipMemcpyAsync(host_stats, ws.pool, static_cast<size_t>(nsizes) * kStatVals * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  return LBM_OK;
}

void fill_balance_stats(const double* host_stats, const int32_t* sizes, int nsizes, lbm_balance_stats* out) {
  for (int k = 0; k < nsizes; ++k) fill_stats(host_stats + static_cast<size_t>(k) * kStatVals, sizes[k], out[k]);
}

size_t balance_stats_doubles() { return static_cast<size_t>(kMaxSizes) * kStatVals; }

int run_balance(const lbm_balance_input& in, const BalanceWs& ws, const int32_t* sizes,
                int nsizes, lbm_balance_stats* out, double* dmaps, const int32_t* windows,
                int nwin, double* wterms, double* term_fields, const lbm_balance_extra* extra) {
  hipStream_t s = static_cast<hipStream_t>(in.stream);
  const int nx = in.nx, ny = in.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  if (int rc = balance_table(in, ws, term_fields != nullptr)) return rc;
  if (term_fields)
    LBM_HIP(hipMemcpyAsync(term_fields, ws.terms, NT * plane * sizeof(double),
                           hipMemcpyDeviceToDevice, s));

  const bool hist = extra && extra->edges;
  const int ne = hist ? extra->nedges : 0;
  const int acc = extra ? extra->accumulate : 0;
  const bool sampled = extra && extra->sample_counts;
  const size_t hslot = 3 * static_cast<size_t>(LBM_MAX_EDGES + 1);  // per size: [3][ne + 1]
  unsigned long long* hall = ws.hist;
  unsigned long long* hsmp = ws.hist + static_cast<size_t>(kMaxSizes) * hslot;
  if (hist) {
    LBM_HIP(hipMemcpyAsync(ws.edges, extra->edges, sizeof(double) * 3 * ne, hipMemcpyHostToDevice, s));
    if (!acc) {
      hipLaunchKernelGGL(k_zero_u64, dim3(256), dim3(256), 0, s, ws.hist, 2 * static_cast<size_t>(kMaxSizes) * hslot);
      LBM_HIP(hipGetLastError());
    }
  }

  SatView v{ws.sat, ws.means, nx, ny, NT, sat_ld(nx)};
  if (out)
    if (int rc = corner_stats(v, ws, sizes, nsizes, dmaps, hist, ne, hall, hslot, acc, s)) return rc;
  if (sampled) {
    size_t off = 0;
    for (int k = 0; k < nsizes; ++k) {
      const size_t cnt = static_cast<size_t>(extra->sample_counts[k]);
      int nb = 0;
      if (cnt > 0) {
        nb = static_cast<int>(std::min<size_t>(kWinMaxBlocks, (cnt + kWinThreads - 1) / kWinThreads));
        if (int rc = launch_windows(hist, v, sizes[k], extra->sample_xy + 2 * off, cnt, nb, nullptr,
                                    ws.partials, ws.edges, ne, hsmp + static_cast<size_t>(k) * hslot, s))
          return rc;
      }
      hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kWinThreads), 0, s, ws.partials, nb,
                         ws.sstats + static_cast<size_t>(k) * kStatVals);
      LBM_HIP(hipGetLastError());
      off += cnt;
    }
    if (nsizes > 0) {
      hipLaunchKernelGGL(k_stats_pool, dim3((3 * nsizes + 63) / 64), dim3(64), 0, s, ws.sstats,
                         ws.pool + static_cast<size_t>(kMaxSizes) * kStatVals, 3 * nsizes, acc);
      LBM_HIP(hipGetLastError());
    }
  }
  if (nwin > 0) {
    LBM_HIP(hipMemcpyAsync(ws.windows, windows, sizeof(int32_t) * 3 * nwin, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_window_terms, dim3((nwin + 63) / 64), dim3(64), 0, s, v, ws.windows, nwin,
                       ws.wterms);
    LBM_HIP(hipGetLastError());
  }
  const size_t sv = static_cast<size_t>(nsizes) * kStatVals;
  // statistics land in fixed-size host arrays (no allocation on this path)
  double st[kMaxSizes * kStatVals], sst[kMaxSizes * kStatVals];
  std::vector<unsigned long long> hh(hist && extra->hist ? nsizes * hslot : 0);
  std::vector<unsigned long long> hs(hist && extra->sample_hist ? nsizes * hslot : 0);
  if (out) LBM_HIP(hipMemcpyAsync(st, ws.pool, sv * sizeof(double), hipMemcpyDeviceToHost, s));
  if (sampled)
    LBM_HIP(hipMemcpyAsync(sst, ws.pool + static_cast<size_t>(kMaxSizes) * kStatVals,
                           sv * sizeof(double), hipMemcpyDeviceToHost, s));
  if (!hh.empty())
    LBM_HIP(hipMemcpyAsync(hh.data(), hall, hh.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  if (!hs.empty())
    LBM_HIP(hipMemcpyAsync(hs.data(), hsmp, hs.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  if (nwin > 0)
    LBM_HIP(hipMemcpyAsync(wterms, ws.wterms, sizeof(double) * LBM_NWVALS * nwin, hipMemcpyDeviceToHost, s));
  LBM_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < nsizes; ++k) {
    if (out) fill_stats(st + static_cast<size_t>(k) * kStatVals, sizes[k], out[k]);
    if (sampled) fill_stats(sst + static_cast<size_t>(k) * kStatVals, sizes[k], extra->sample_out[k]);
    auto unpack = [&](const std::vector<unsigned long long>& src, int64_t* dst) {
      for (int q = 0; q < 3; ++q)
        for (int i = 0; i <= ne; ++i)
          dst[(static_cast<size_t>(k) * 3 + q) * (ne + 1) + i] =
              static_cast<int64_t>(src[static_cast<size_t>(k) * hslot + q * (ne + 1) + i]);
    };
    if (!hh.empty()) unpack(hh, extra->hist);
    if (!hs.empty()) unpack(hs, extra->sample_hist);
  }
  return LBM_OK;
}

}  // namespace lbm
