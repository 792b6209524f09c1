// Entropic lattice Boltzmann step (Sec. 1: the H-functional of Eq. 6 and the
// effective relaxation time tau_eff = 2 tau0 / alpha) for gfx950.
//
// Per site, in FP64 whatever the storage type: the minimiser of H at the
// site's rho and rho u in closed form,
//   f^eq_l = t_l rho prod_a (2 - s_a) ((2 u_a + s_a) / (1 - u_a))^{c_la},  s_a = sqrt(1 + 3 u_a^2),
// delta = f^eq - f, and alpha the root alpha > 1 of the entropy equality
// H(f + alpha delta) = H(f), found by Newton's method inside a bracket
// [1, alpha_max) kept by bisection (alpha_max: the largest step keeping every
// population positive), started from the root of the gain expanded to fourth
// order in delta / f around alpha = 2.  The entropy gain is evaluated as
//   g(a) = sum_l f_l phi(a delta_l / f_l) - a sum_l delta_l log1p(delta_l / f_l),
//   phi(t) = (1 + t) log1p(t) - t,
// which is H(f + a delta) - H(f) with the first-order terms cancelled
// analytically (delta conserves mass and momentum and log(f^eq / t) is affine
// in c), so it keeps its relative accuracy close to equilibrium.  Then
// f* = f + alpha beta delta, beta = 1 / (2 tau0), pull-streamed like the BGK
// step (one site per thread, the same tiling).
#include <hip/hip_runtime.h>

#include <cmath>

#include "lbm_internal.h"
#include "lbm_site.h"

namespace lbm {
namespace {

using namespace step_detail;

// below this max_l |delta_l| / f_l the site counts as at equilibrium: alpha = 2
constexpr double kNearEq = 1e-8;
// below this max_l |delta_l| / f_l the gain is evaluated as its power series in
// x = delta / f, truncated after x^kSeriesN: for a <= 3 the first omitted term
// is below (3 * 0.015)^(kSeriesN + 1) / kSeriesN ~ 1e-17 of the leading one
constexpr double kSeriesMax = 0.015;
constexpr int kSeriesN = 12;
// workgroups of at most this many threads, so the FP64 site state stays in registers
constexpr int kEntropicMaxThreads = 256;

// 1/x in FP64 (x > 0, normal): the hardware estimate refined by two Newton steps,
// r <- r + r (1 - x r), to within an ulp or two of the quotient at a fraction of
// the instructions of a division.
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return r;
}

struct EntropicSite {
  double f[9];
  double x[9];  // delta / f, delta = f^eq - f
  double rho, ux, uy;
};

template <typename T>
__device__ __forceinline__ void entropic_site(const T (&d)[9], EntropicSite& s) {
  double drho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const double dv = double(d[l]);
    s.f[l] = wq(l) + dv;
    drho += dv;
    jx += cxq(l) * dv;
    jy += cyq(l) * dv;
  }
  s.rho = 1.0 + drho;
  const double ir = rcp64(s.rho);
  s.ux = jx * ir;
  s.uy = jy * ir;
  const double sx = sqrt(1.0 + 3.0 * s.ux * s.ux), sy = sqrt(1.0 + 3.0 * s.uy * s.uy);
  // z_a = (2 u_a + s_a) / (1 - u_a) and its inverse
  const double nx_ = 2.0 * s.ux + sx, dx_ = 1.0 - s.ux, ny_ = 2.0 * s.uy + sy, dy_ = 1.0 - s.uy;
  const double zx = nx_ * rcp64(dx_), izx = dx_ * rcp64(nx_);
  const double zy = ny_ * rcp64(dy_), izy = dy_ * rcp64(ny_);
  const double base = s.rho * (2.0 - sx) * (2.0 - sy);
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    double e = wq(l) * base;
    if (cxq(l) == 1) e *= zx;
    if (cxq(l) == -1) e *= izx;
    if (cyq(l) == 1) e *= zy;
    if (cyq(l) == -1) e *= izy;
    s.x[l] = (e - s.f[l]) * rcp64(s.f[l]);
  }
}

// g(a) and g'(a) for the site; c1 = sum delta log1p(delta / f).
__device__ __forceinline__ double entropy_gain(const EntropicSite& s, double c1, double a, double& dg) {
  double g = 0.0, gd = 0.0;
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const double t = a * s.x[l];
    const double lp = log1p(t);
    g += s.f[l] * ((1.0 + t) * lp - t);
    gd += s.f[l] * s.x[l] * lp;
  }
  dg = gd - c1;
  return g - a * c1;
}

// The gain as a power series: with t = a x, (1 + t) log1p(t) - t =
// sum_{n>=2} (-1)^n t^n / (n (n - 1)) and x log1p(x) = sum_{n>=2} (-1)^n x^n / (n - 1), so
//   g(a) = P(a) - a Q,  P(a) = sum_n (-1)^n S_n a^n / (n (n - 1)),  Q = sum_n (-1)^n S_n / (n - 1),
// S_n = sum_l f_l x_l^n; g'(a) = P'(a) - Q.  cp[n] = (-1)^n S_n / (n (n - 1)).
struct GainSeries {
  double cp[kSeriesN + 1];
  double q;
  __device__ __forceinline__ double eval(double a, double& dg) const {
    double p = cp[kSeriesN], dp = kSeriesN * cp[kSeriesN];
#pragma unroll
    for (int n = kSeriesN - 1; n >= 2; --n) {
      p = p * a + cp[n];
      dp = dp * a + n * cp[n];
    }
    // p = sum cp[n] a^(n-2), dp = sum n cp[n] a^(n-2)
    const double a2 = a * a;
    dg = dp * a - q;
    return p * a2 - a * q;
  }
};

__device__ __forceinline__ void gain_series(const EntropicSite& s, GainSeries& gs) {
  double sn[kSeriesN + 1];
#pragma unroll
  for (int n = 0; n <= kSeriesN; ++n) sn[n] = 0.0;
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const double x = s.x[l];
    double p = s.f[l] * x * x;
#pragma unroll
    for (int n = 2; n <= kSeriesN; ++n) {
      sn[n] += p;
      p *= x;
    }
  }
  gs.q = 0.0;
#pragma unroll
  for (int n = 2; n <= kSeriesN; ++n) {
    const double sg = (n & 1) ? -sn[n] : sn[n];
    const double inn = 1.0 / (n * (n - 1.0)), in1 = 1.0 / (n - 1.0);  // constants after unrolling
    gs.cp[n] = sg * inn;
    gs.q += sg * in1;
  }
}

// Newton's method on g(a) = 0 in the bracket [lo, hi], from a; with SERIES the
// gain is the power series gs, else the logarithm form with c1.  A Newton step
// below 1e-10 a ends it (quadratic convergence: the iterate is then within
// ~1e-20 of the root), whether or not it stays inside the bracket: a step that
// lands on the bracket's end (the gain's sign at the root decided by rounding)
// used to fall back to bisection down to a 1e-15 bracket, up to 50 iterations,
// and a wavefront runs as long as its slowest site.  Steps leaving the bracket
// otherwise are replaced by bisection, which ends at a 1e-15 bracket.
template <bool SERIES>
__device__ __forceinline__ double newton_alpha(const EntropicSite& s, const GainSeries& gs, double c1,
                                               double a, double lo, double hi) {
  auto gain = [&](double x, double& dg) {
    if constexpr (SERIES)
      return gs.eval(x, dg);
    else
      return entropy_gain(s, c1, x, dg);
  };
  double dg;
  double ga = gain(a, dg);
  if (ga < 0.0) {
    double dgh;
    if (gain(hi, dgh) < 0.0) return hi;  // no root below the positivity limit
    lo = a;
  } else {
    hi = a;
  }
  for (int it = 0; it < 64; ++it) {
    const double step = ga / dg;
    if (fabs(step) <= 1e-10 * a) return a - step;
    double an = a - step;
    if (!(an > lo && an < hi)) {
      an = 0.5 * (lo + hi);
      if (hi - lo <= 1e-15 * hi) return an;
    }
    a = an;
    ga = gain(a, dg);
    if (ga < 0.0)
      lo = a;
    else
      hi = a;
  }
  return a;
}

__device__ double entropic_alpha(const EntropicSite& s) {
  double mr = 0.0, xmin = 0.0;
  double s2 = 0.0, s3 = 0.0, s4 = 0.0;  // sum f x^k: the expansion of the gain in x = delta / f
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const double x = s.x[l];
    mr = fmax(mr, fabs(x));
    xmin = fmin(xmin, x);
    const double fx2 = s.f[l] * x * x;
    s2 += fx2;
    s3 += fx2 * x;
    s4 += fx2 * x * x;
  }
  if (mr < kNearEq) return 2.0;
  const double amax = xmin < 0.0 ? -1.0 / xmin : 1e300;  // every f + a delta > 0 below it
  // close to equilibrium the series replaces the logarithms, for a <= 3
  const bool series = mr < kSeriesMax;
  double lo = 1.0, hi = amax < 1e300 ? amax * (1.0 - 1e-12) : 1e6;
  if (series) hi = fmin(hi, 3.0);  // the root lies within 2 +- O(mr); the series holds up to 3
  // start from the root of the gain expanded to fourth order around a = 2:
  // g(2 + e) / (2 + e) = e S2 / 2 - S3 / 6 + S4 / 3 + ... = 0
  // (the expansion is only trusted close to 2: far from equilibrium start at 2)
  double a = 2.0 + (s3 - 2.0 * s4) / (3.0 * s2);
  if (!(fabs(a - 2.0) < 0.25 && a > lo && a < hi)) a = 2.0 < hi ? 2.0 : 0.5 * (lo + hi);
  GainSeries gs;
  if (series) {
    gain_series(s, gs);
    return newton_alpha<true>(s, gs, 0.0, a, lo, hi);
  }
  double c1 = 0.0;
#pragma unroll
  for (int l = 0; l < 9; ++l) c1 += s.f[l] * s.x[l] * log1p(s.x[l]);
  return newton_alpha<false>(s, gs, c1, a, lo, hi);
}

template <typename T, bool NT>
__global__ void __launch_bounds__(kEntropicMaxThreads) k_elbm_step(StepParams p, int tiles_x, int total,
                                                                    int per_xcd, int ry) {
  const int b = blockIdx.x;
  const int tile = (b & 7) * per_xcd + (b >> 3);
  if (tile >= total) return;
  const int tx = tile % tiles_x;
  const int ty = tile / tiles_x;
  const int x = tx * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const int ybase = (ty * blockDim.y + threadIdx.y) * ry;
  const int nx = p.nx, ny = p.ny;
  const T* __restrict__ src = static_cast<const T*>(p.src);
  T* __restrict__ dst = static_cast<T*>(p.dst);
  const double beta = 0.5 * p.omega;  // 1 / (2 tau0)
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
    EntropicSite s;
    entropic_site<T>(di, s);
    const double ab = entropic_alpha(s) * beta;
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      const T o = T(double(di[l]) + ab * (s.f[l] * s.x[l]));
      T* q = dst + l * p.ps + static_cast<size_t>(y) * p.rs + x;
      if constexpr (NT) __builtin_nontemporal_store(o, q);
      else *q = o;
    }
    if (p.h_rho) {
      const size_t i = static_cast<size_t>(y) * nx + x;
      p.h_rho[i] = s.rho;
      p.h_ux[i] = s.ux;
      p.h_uy[i] = s.uy;
    }
  }
}

// alpha and nu_eff = c_s^2 (2 tau0 / alpha - 1/2) of the current populations.
template <typename T>
__global__ void __launch_bounds__(256) k_elbm_relax(const T* __restrict__ pop, size_t ps, size_t rs, int nx,
                                                    int ny, double tau0, double* alpha, double* nu) {
  const size_t plane = static_cast<size_t>(nx) * ny;
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < plane; i += size_t(gridDim.x) * 256) {
    const int x = static_cast<int>(i % nx), y = static_cast<int>(i / nx);
    T d[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      int xs = x - cxq(l), ys = y - cyq(l);
      xs += xs < 0 ? nx : 0;
      xs -= xs >= nx ? nx : 0;
      ys += ys < 0 ? ny : 0;
      ys -= ys >= ny ? ny : 0;
      d[l] = pop[l * ps + static_cast<size_t>(ys) * rs + xs];
    }
    EntropicSite s;
    entropic_site<T>(d, s);
    const double a = entropic_alpha(s);
    if (alpha) alpha[i] = a;
    if (nu) nu[i] = (2.0 * tau0 / a - 0.5) / 3.0;
  }
}

__global__ void k_fill_relax(size_t n, double a, double v, double* alpha, double* nu) {
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256) {
    if (alpha) alpha[i] = a;
    if (nu) nu[i] = v;
  }
}

template <typename T>
int launch_t(const StepParams& p, const lbm_tile& t, hipStream_t s) {
  const int tiles_x = (p.nx + t.bx - 1) / t.bx;
  const int rows_per_tile = t.by * t.ry;
  const int tiles_y = (p.ny + rows_per_tile - 1) / rows_per_tile;
  const int total = tiles_x * tiles_y;
  const int per_xcd = (total + 7) / 8;
  if (t.nt)
    hipLaunchKernelGGL((k_elbm_step<T, true>), dim3(per_xcd * 8), dim3(t.bx, t.by), 0, s, p, tiles_x, total,
                       per_xcd, t.ry);
  else
    hipLaunchKernelGGL((k_elbm_step<T, false>), dim3(per_xcd * 8), dim3(t.bx, t.by), 0, s, p, tiles_x, total,
                       per_xcd, t.ry);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

}  // namespace

bool entropic_tile_ok(const lbm_tile& t, int nx, int ny) {
  return edm_tile_ok(t, nx, ny) && t.bx * t.by <= kEntropicMaxThreads;
}

int entropic_step(int dtype, const StepParams& p, const lbm_tile& t, hipStream_t s) {
  if (!entropic_tile_ok(t, p.nx, p.ny)) return fail(LBM_E_INVALID, "invalid launch shape for the entropic step");
  return dtype == LBM_F64 ? launch_t<double>(p, t, s) : launch_t<float>(p, t, s);
}

int relaxation_fields(int dtype, bool entropic, const void* pop, PopLayout lay, int nx, int ny, double tau0,
                      double* alpha, double* nu, hipStream_t s) {
  const size_t n = static_cast<size_t>(nx) * ny;
  const int g = static_cast<int>(n / 256 + 1 < 4096 ? n / 256 + 1 : 4096);
  if (!entropic)
    hipLaunchKernelGGL(k_fill_relax, dim3(g), dim3(256), 0, s, n, 2.0, (tau0 - 0.5) / 3.0, alpha, nu);
  else if (dtype == LBM_F64)
    hipLaunchKernelGGL(k_elbm_relax<double>, dim3(g), dim3(256), 0, s, static_cast<const double*>(pop), lay.ps,
                       lay.rs, nx, ny, tau0, alpha, nu);
  else
    hipLaunchKernelGGL(k_elbm_relax<float>, dim3(g), dim3(256), 0, s, static_cast<const float*>(pop), lay.ps,
                       lay.rs, nx, ny, tau0, alpha, nu);
  LBM_HIP(hipGetLastError());
  return LBM_OK;
}

}  // namespace lbm
