// Device helpers shared by the LDS-resident dense kernels (one workgroup of
// NT = 256 threads per node).
#pragma once

#include "ht_internal.h"

namespace ht {

constexpr int DNT = 256;  // threads per workgroup of the dense kernels

// Sum / max over the workgroup: wave shuffles, then one LDS stage.
// red needs DNT/64 doubles; two barriers.
__device__ __forceinline__ double wg_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < DNT / 64; ++i) r += red[i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double wg_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int i = 1; i < DNT / 64; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

// Binary exponent e with x = m 2^e, 0.5 <= m < 1 (0 for x = 0 or non-finite).
__device__ __forceinline__ int exp2_of(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 0;
  int e;
  frexp(x, &e);
  return e;
}

}  // namespace ht
