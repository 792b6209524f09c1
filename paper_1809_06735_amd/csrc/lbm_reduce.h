// Wave and workgroup reductions in FP64, fixed order (the same inputs give the
// same bits on every run).
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {
namespace reduce_detail {

constexpr int kRedThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Reduce 7 per-thread values (sum x4, max, min, sum) over a workgroup of
// kRedThreads threads; thread 0 writes them to out[0..6] and 0 to out[7].
__device__ inline void block_reduce7(double (&v)[7], double* out) {
  __shared__ double sh[kRedThreads / 64][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double r[7];
  r[0] = wave_sum(v[0]);
  r[1] = wave_sum(v[1]);
  r[2] = wave_sum(v[2]);
  r[3] = wave_sum(v[3]);
  r[4] = wave_max(v[4]);
  r[5] = wave_min(v[5]);
  r[6] = wave_sum(v[6]);
  if (lane == 0)
    for (int k = 0; k < 7; ++k) sh[wv][k] = r[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double a[7];
    for (int k = 0; k < 7; ++k) a[k] = sh[0][k];
    for (int w = 1; w < kRedThreads / 64; ++w) {
      a[0] += sh[w][0];
      a[1] += sh[w][1];
      a[2] += sh[w][2];
      a[3] += sh[w][3];
      a[4] = fmax(a[4], sh[w][4]);
      a[5] = fmin(a[5], sh[w][5]);
      a[6] += sh[w][6];
    }
    for (int k = 0; k < 7; ++k) out[k] = a[k];
    out[7] = 0.0;
  }
}

}  // namespace reduce_detail
}  // namespace lbm
