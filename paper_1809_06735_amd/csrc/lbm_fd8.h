// 8th-order centred differences (Eq. 18) on periodic FP64 fields, shared by the
// balance and the adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace lbm {
namespace fd8 {

__device__ __forceinline__ int wrap_add(int i, int m, int n) {
  int j = i + m;
  j -= j >= n ? n : 0;
  j += j < 0 ? n : 0;
  return j;
}

// Eq. 18 applied to a value accessor g(x, y) along x or y.
template <class G>
__device__ __forceinline__ double fd8_x(const G& g, int x, int y, int nx) {
  const double d1 = g(wrap_add(x, 1, nx), y) - g(wrap_add(x, -1, nx), y);
  const double d2 = g(wrap_add(x, 2, nx), y) - g(wrap_add(x, -2, nx), y);
  const double d3 = g(wrap_add(x, 3, nx), y) - g(wrap_add(x, -3, nx), y);
  const double d4 = g(wrap_add(x, 4, nx), y) - g(wrap_add(x, -4, nx), y);
  return (4.0 * d1 - d2 + (4.0 / 21.0) * d3 - (1.0 / 56.0) * d4) / 5.0;
}
template <class G>
__device__ __forceinline__ double fd8_y(const G& g, int x, int y, int ny) {
  const double d1 = g(x, wrap_add(y, 1, ny)) - g(x, wrap_add(y, -1, ny));
  const double d2 = g(x, wrap_add(y, 2, ny)) - g(x, wrap_add(y, -2, ny));
  const double d3 = g(x, wrap_add(y, 3, ny)) - g(x, wrap_add(y, -3, ny));
  const double d4 = g(x, wrap_add(y, 4, ny)) - g(x, wrap_add(y, -4, ny));
  return (4.0 * d1 - d2 + (4.0 / 21.0) * d3 - (1.0 / 56.0) * d4) / 5.0;
}

struct F1 {
  const double* __restrict__ a;
  int nx;
  __device__ double operator()(int x, int y) const { return a[static_cast<size_t>(y) * nx + x]; }
};
struct F2 {  // a * b
  const double* __restrict__ a;
  const double* __restrict__ b;
  int nx;
  __device__ double operator()(int x, int y) const {
    const size_t i = static_cast<size_t>(y) * nx + x;
    return a[i] * b[i];
  }
};
struct FSum2 {  // a * b + c * d
  const double* __restrict__ a;
  const double* __restrict__ b;
  const double* __restrict__ c;
  const double* __restrict__ d;
  int nx;
  __device__ double operator()(int x, int y) const {
    const size_t i = static_cast<size_t>(y) * nx + x;
    return a[i] * b[i] + c[i] * d[i];
  }
};
struct FDiv {  // a / b
  const double* __restrict__ a;
  const double* __restrict__ b;
  int nx;
  __device__ double operator()(int x, int y) const {
    const size_t i = static_cast<size_t>(y) * nx + x;
    return a[i] / b[i];
  }
};

}  // namespace fd8
}  // namespace lbm
