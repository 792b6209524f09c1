// Kinetic-energy spectrum of a periodic velocity field (the shell-summed spectra
// of Sec. 4, Fig. 5 and Sec. 5, Fig. 10) for gfx950.
//
// With z = u_x + i u_y and Z its discrete Fourier transform divided by nx ny,
// the Fourier-series coefficients of the components are
// u^_x(k) = (Z(k) + conj Z(-k)) / 2 and u^_y(k) = (Z(k) - conj Z(-k)) / (2i), so
// |u^_x|^2 + |u^_y|^2 = (|Z(k)|^2 + |Z(-k)|^2) / 2, and since a shell maps onto
// itself under k -> -k, E(s) = 1/2 sum_{k in s} |Z(k)|^2: one complex 2D FFT.
//
// Passes (FP64 complex throughout): pack z and transform every row in LDS
// (radix-2, decimation in time, bit-reversed load, twiddles from a table of
// exp(-2 pi i k / nmax)); transpose through LDS tiles; transform the rows of
// the transpose (the columns); then one workgroup per shell adds 1/2 |Z|^2
// over the shell's wavevectors in a fixed order (no atomics: the spectrum is
// bitwise reproducible).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int kFftMax = 4096;
constexpr int kFftThreads = 256;

__global__ void __launch_bounds__(256) k_twiddles(double2* __restrict__ tw, int nmax) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nmax / 2) return;
  double s, c;
  sincospi(-2.0 * k / nmax, &s, &c);
  tw[k] = make_double2(c, s);
}

// One row of n = 2^logn values per workgroup, transformed in place in LDS.
// PACK: the row is (ux + i uy) of FP64 fields, else complex data in `d`.
template <bool PACK>
__global__ void __launch_bounds__(kFftThreads) k_fft_rows(const double* __restrict__ ux,
                                                          const double* __restrict__ uy,
                                                          double2* __restrict__ data, int n, int logn,
                                                          const double2* __restrict__ tw, int nmax) {
  __shared__ double2 sh[kFftMax];
  const size_t row = blockIdx.x;
  double2* d = data + row * n;
  for (int x = threadIdx.x; x < n; x += kFftThreads) {
    const double2 v = PACK ? make_double2(ux[row * n + x], uy[row * n + x]) : d[x];
    sh[__brev(static_cast<unsigned>(x)) >> (32 - logn)] = v;
  }
  __syncthreads();
  for (int s = 1; s <= logn; ++s) {
    const int h = 1 << (s - 1);        // half the butterfly span m = 2h
    const int step = nmax >> s;         // exp(-2 pi i j / m) = tw[j nmax / m]
    for (int b = threadIdx.x; b < n / 2; b += kFftThreads) {
      const int j = b & (h - 1);
      const int i0 = ((b >> (s - 1)) << s) + j, i1 = i0 + h;
      const double2 w = tw[j * step];
      const double2 a = sh[i0], c = sh[i1];
      const double2 t = make_double2(w.x * c.x - w.y * c.y, w.x * c.y + w.y * c.x);
      sh[i0] = make_double2(a.x + t.x, a.y + t.y);
      sh[i1] = make_double2(a.x - t.x, a.y - t.y);
    }
    __syncthreads();
  }
  for (int x = threadIdx.x; x < n; x += kFftThreads) d[x] = sh[x];
}

// b[x][y] = a[y][x] for a [ny][nx], through 32 x 32 tiles.
__global__ void __launch_bounds__(256) k_transpose(const double2* __restrict__ a, double2* __restrict__ b,
                                                   int nx, int ny) {
  __shared__ double2 t[32][33];
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
  for (int j = threadIdx.y; j < 32; j += 8) {
    const int x = x0 + threadIdx.x, y = y0 + j;
    if (x < nx && y < ny) t[j][threadIdx.x] = a[static_cast<size_t>(y) * nx + x];
  }
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += 8) {
    const int y = y0 + threadIdx.x, x = x0 + j;
    if (x < nx && y < ny) b[static_cast<size_t>(x) * ny + y] = t[threadIdx.x][j];
  }
}

// Largest f >= 0 with 4 f^2 <= q (q >= 0).
__device__ __forceinline__ long long isqrt4(long long q) {
  long long f = static_cast<long long>(sqrt(static_cast<double>(q) / 4.0));
  while (f > 0 && 4 * f * f > q) --f;
  while (4 * (f + 1) * (f + 1) <= q) ++f;
  return f;
}

// z [nx][ny] after both passes: row index = x frequency, column = y frequency.
// One workgroup per shell s gathers the shell's wavevectors, those with
// (2s - 1)^2 <= 4 |k|^2 < (2s + 1)^2: thread t takes the x frequencies
// fx = -s + t, -s + t + 256, ... (within the grid's signed range), and for each
// the y frequencies of the annulus, two contiguous runs +-[fy_lo, fy_hi], in
// increasing order; the threads' sums are added by a fixed tree.  No atomics:
// the result does not depend on scheduling.
__global__ void __launch_bounds__(256) k_shells(const double2* __restrict__ z, int nx, int ny, double scale,
                                                double* __restrict__ spec) {
  __shared__ double wsum[4];
  const long long sh = blockIdx.x;
  const long long qlo = sh > 0 ? (2 * sh - 1) * (2 * sh - 1) : 0;  // 4|k|^2 >= qlo
  const long long qhi = (2 * sh + 1) * (2 * sh + 1) - 1;           // 4|k|^2 <= qhi
  const long long fxa = max(-sh, static_cast<long long>(-(nx / 2)));
  const long long fxb = min(sh, static_cast<long long>(nx - nx / 2 - 1));
  const long long fya = -(ny / 2), fyb = ny - ny / 2 - 1;
  double acc = 0.0;
  for (long long fx = fxa + threadIdx.x; fx <= fxb; fx += 256) {
    const long long a4 = 4 * fx * fx;
    if (a4 > qhi) continue;
    const long long hi = isqrt4(qhi - a4);                       // |fy| <= hi
    const long long lo = qlo > a4 ? isqrt4(qlo - a4 - 1) + 1 : 0;  // |fy| >= lo
    if (lo > hi) continue;
    const double2* row = z + static_cast<size_t>(fx < 0 ? fx + nx : fx) * ny;
    // negative y frequencies -hi .. -lo (skipping 0), then lo .. hi
    for (long long fy = max(-hi, fya); fy <= min(-max(lo, 1LL), fyb); ++fy) {
      const double2 v = row[fy + ny];
      acc += v.x * v.x + v.y * v.y;
    }
    for (long long fy = max(lo, fya); fy <= min(hi, fyb); ++fy) {
      const double2 v = row[fy];
      acc += v.x * v.x + v.y * v.y;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) spec[blockIdx.x] = 0.5 * scale * ((wsum[0] + wsum[1]) + (wsum[2] + wsum[3]));
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Shells that can hold a wavevector: 0 .. shell of (nx/2, ny/2).
int useful_shells(int nx, int ny) {
  const long long k2 = static_cast<long long>(nx / 2) * (nx / 2) + static_cast<long long>(ny / 2) * (ny / 2);
  int s = static_cast<int>(std::sqrt(static_cast<double>(k2)) + 0.5);
  while (static_cast<long long>(2 * s + 1) * (2 * s + 1) <= 4 * k2) ++s;
  return s + 1;
}

}  // namespace

bool spectrum_size_ok(int nx, int ny) {
  auto pow2 = [](int n) { return n >= 16 && n <= kFftMax && (n & (n - 1)) == 0; };
  return pow2(nx) && pow2(ny);
}

size_t spectrum_ws_bytes(int nx, int ny) {
  Carver c(nullptr, 0);
  c.take<double2>(2 * static_cast<size_t>(nx) * ny);
  c.take<double2>(std::max(nx, ny) / 2);
  c.take<double>(useful_shells(nx, ny));
  return c.used + 256;
}

int run_spectrum(int nx, int ny, const double* ux, const double* uy, void* ws, size_t ws_bytes,
                 double* spectrum, int nshells, hipStream_t s) {
  if (!spectrum_size_ok(nx, ny))
    return fail(LBM_E_UNSUPPORTED, "spectrum needs power-of-two extents in [16, %d] (got %d x %d)", kFftMax,
                nx, ny);
  if (nshells < 1 || nshells > LBM_MAX_SHELLS)
    return fail(LBM_E_INVALID, "nshells must be in [1, %d]", LBM_MAX_SHELLS);
  if (!ux || !uy || !spectrum) return fail(LBM_E_INVALID, "NULL field or output");
  if (ws_bytes < spectrum_ws_bytes(nx, ny)) return fail(LBM_E_NOMEM, "spectrum workspace too small");
  Carver c(ws, ws_bytes);
  const int nmax = std::max(nx, ny);
  const int ns = std::min(nshells, useful_shells(nx, ny));  // shells past these are empty
  double2* a = c.take<double2>(static_cast<size_t>(nx) * ny);
  double2* b = c.take<double2>(static_cast<size_t>(nx) * ny);
  double2* tw = c.take<double2>(nmax / 2);
  double* spec = c.take<double>(useful_shells(nx, ny));
  hipLaunchKernelGGL(k_twiddles, dim3((nmax / 2 + 255) / 256), dim3(256), 0, s, tw, nmax);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_fft_rows<true>, dim3(ny), dim3(kFftThreads), 0, s, ux, uy, a, nx, ilog2(nx), tw, nmax);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_transpose, dim3((nx + 31) / 32, (ny + 31) / 32), dim3(32, 8), 0, s, a, b, nx, ny);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_fft_rows<false>, dim3(nx), dim3(kFftThreads), 0, s, nullptr, nullptr, b, ny, ilog2(ny),
                     tw, nmax);
  LBM_HIP(hipGetLastError());
  const double inv = 1.0 / (static_cast<double>(nx) * ny);
  hipLaunchKernelGGL(k_shells, dim3(ns), dim3(256), 0, s, b, nx, ny, inv * inv, spec);
  LBM_HIP(hipGetLastError());
  LBM_HIP(hipMemcpyAsync(spectrum, spec, ns * sizeof(double), hipMemcpyDeviceToHost, s));
  LBM_HIP(hipStreamSynchronize(s));
  for (int k = ns; k < nshells; ++k) spectrum[k] = 0.0;
  return LBM_OK;
}

}  // namespace lbm
