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

// 1 / x from the hardware reciprocal refined by two Newton steps (within an
// ulp or two of the correctly rounded quotient; x finite and nonzero).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// 1 / sqrt(x) for x > 0: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// Value of v in lane src (src uniform).
__device__ __forceinline__ double lane_val(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// DPP move of a double within rows of 16 lanes (CTRL: a DPP control code
// whose source lane always lies in the row, so every lane is written and
// bound_ctrl changes nothing).  With bound_ctrl set the compiler needs no
// initialised destination, and row_newbcast becomes one v_mov_b64_dpp.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xF, 0xF, true);
}

// Lane j's value (j a compile-time constant after unrolling) to every lane of
// its 16-lane DPP row: row_newbcast, a VALU move with no scalar round trip.
__device__ __forceinline__ double row16_bcast(double v, int j) {
  switch (j & 15) {
    case 0: return dpp_f64<0x150>(v);
    case 1: return dpp_f64<0x151>(v);
    case 2: return dpp_f64<0x152>(v);
    case 3: return dpp_f64<0x153>(v);
    case 4: return dpp_f64<0x154>(v);
    case 5: return dpp_f64<0x155>(v);
    case 6: return dpp_f64<0x156>(v);
    case 7: return dpp_f64<0x157>(v);
    case 8: return dpp_f64<0x158>(v);
    case 9: return dpp_f64<0x159>(v);
    case 10: return dpp_f64<0x15A>(v);
    case 11: return dpp_f64<0x15B>(v);
    case 12: return dpp_f64<0x15C>(v);
    case 13: return dpp_f64<0x15D>(v);
    case 14: return dpp_f64<0x15E>(v);
    default: return dpp_f64<0x15F>(v);
  }
}

// Sum over the 16 lanes of a DPP row, returned to every lane of the row:
// swap neighbours, swap pairs (quad permutations), then the half-row and
// row mirrors join quads into eights and eights into sixteen.
__device__ __forceinline__ double row16_sum(double s) {
  s += dpp_f64<0xB1>(s);    // quad_perm [1,0,3,2]
  s += dpp_f64<0x4E>(s);    // quad_perm [2,3,0,1]
  s += dpp_f64<0x141>(s);   // row_half_mirror
  s += dpp_f64<0x140>(s);   // row_mirror
  return s;
}

// Binary exponent e with x = m 2^e, 0.5 <= m < 1 (0 for x = 0 or non-finite).
__device__ __forceinline__ int exp2_of(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 0;
  int e;
  frexp(x, &e);
  return e;
}

}  // namespace ht
