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
// the transpose (the columns); add 1/2 |Z|^2 into the shells in LDS and then
// into the device spectrum.  The shell sums use FP64 atomics, so the last bits
// of a shell's sum depend on the order in which workgroups finish.
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

__global__ void k_zero_f64(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Signed frequency of FFT index i of length n (n/2 maps to -n/2).
__device__ __forceinline__ int signed_freq(int i, int n) { return i < n / 2 ? i : i - n; }

// Shell s with (2s - 1)^2 <= 4 k2 < (2s + 1)^2 (s = 0 for k2 = 0).
__device__ __forceinline__ int shell_of(long long k2) {
  int s = static_cast<int>(floor(sqrt(static_cast<double>(k2)) + 0.5));
  const long long q = 4 * k2;
  if (s > 0 && static_cast<long long>(2 * s - 1) * (2 * s - 1) > q) --s;
  if (static_cast<long long>(2 * s + 1) * (2 * s + 1) <= q) ++s;
  return s;
}

// z [nx][ny] after both passes: row index = x frequency, column = y frequency.
__global__ void __launch_bounds__(256) k_shells(const double2* __restrict__ z, int nx, int ny, int nshells,
                                                double scale, double* __restrict__ spec) {
  extern __shared__ double bins[];
  for (int s = threadIdx.x; s < nshells; s += blockDim.x) bins[s] = 0.0;
  __syncthreads();
  const size_t total = static_cast<size_t>(nx) * ny;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < total; i += size_t(gridDim.x) * blockDim.x) {
    const int kxi = static_cast<int>(i / ny), kyi = static_cast<int>(i % ny);
    const long long fx = signed_freq(kxi, nx), fy = signed_freq(kyi, ny);
    const int s = shell_of(fx * fx + fy * fy);
    if (s < nshells) {
      const double2 v = z[i];
      atomicAdd(&bins[s], 0.5 * scale * (v.x * v.x + v.y * v.y));
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < nshells; s += blockDim.x)
    if (bins[s] != 0.0) atomicAdd(&spec[s], bins[s]);
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
  hipLaunchKernelGGL(k_zero_f64, dim3((ns + 255) / 256), dim3(256), 0, s, spec, ns);
  LBM_HIP(hipGetLastError());
  const double inv = 1.0 / (static_cast<double>(nx) * ny);
  const size_t total = static_cast<size_t>(nx) * ny;
  const int g = static_cast<int>(std::min<size_t>(1024, (total + 255) / 256));
  hipLaunchKernelGGL(k_shells, dim3(g), dim3(256), ns * sizeof(double), s, b, nx, ny, ns, inv * inv, spec);
  LBM_HIP(hipGetLastError());
  LBM_HIP(hipMemcpyAsync(spectrum, spec, ns * sizeof(double), hipMemcpyDeviceToHost, s));
  LBM_HIP(hipStreamSynchronize(s));
  for (int k = ns; k < nshells; ++k) spectrum[k] = 0.0;
  return LBM_OK;
}

}  // namespace lbm
