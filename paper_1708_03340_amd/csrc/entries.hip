// Entry evaluation (Section 3.1), level by level for m multi-indices at once.
// Leaves gather row i_mu of U_mu; inner nodes apply eq. (transfermult) as a
// float64 GEMM whose left operand is the row-wise Khatri-Rao product of the
// son rows (gemm.hip, Khatri-Rao mode); the root applies the root formula the
// same way with k_D = 1.  Every node's rows are divided by a power of two per
// index and the exponents are carried up, so entries of tensors whose norm
// exceeds the float64 range are still exact in their mantissa.
#include "ht_internal.h"

namespace ht {
namespace {

__device__ __forceinline__ int exp2_of(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 0;
  int e;
  frexp(x, &e);
  return e;
}

// one wave64 per (node, index): gather the leaf row
__global__ void gather_kernel(const EntryNode* __restrict__ nodes, int64_t m, const int32_t* __restrict__ idx,
                              int d) {
  const EntryNode& nd = nodes[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= m) return;
  const int64_t row = idx[i * d + nd.mode];
  for (int c = lane; c < nd.k; c += 64) {
    const int64_t off = row + (int64_t)c * nd.ld;
    nd.rows[i * nd.k + c] = nd.tdtype == F64 ? reinterpret_cast<const double*>(nd.U)[off]
                                             : (double)reinterpret_cast<const float*>(nd.U)[off];
  }
}

// one wave64 per (node, index): rows[i] *= 2^-e, expo[i] = e (+ son exponents)
__global__ void normalize_kernel(const EntryNode* __restrict__ nodes, int64_t m) {
  const EntryNode& nd = nodes[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= m) return;
  double* r = nd.rows + i * nd.k;
  double mx = 0.0;
  for (int c = lane; c < nd.k; c += 64) mx = fmax(mx, fabs(r[c]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  const int e = exp2_of(mx);
  for (int c = lane; c < nd.k; c += 64) r[c] = ldexp(r[c], -e);
  if (lane == 0) {
    int base = 0;
    if (nd.expo1) base += nd.expo1[i];
    if (nd.expo2) base += nd.expo2[i];
    nd.expo[i] = base + e;
  }
}

__global__ void finish_kernel(const double* vals, const int32_t* expo, int64_t m, long long scale, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  long long e = (long long)expo[i] + scale;
  if (e > 4000) e = 4000;
  if (e < -4000) e = -4000;
  out[i] = ldexp(vals[i], (int)e);
}

}  // namespace

hipError_t launch_entry_gather(const EntryNode* nodes, int n, int64_t m, const int32_t* idx, int d, int,
                               hipStream_t s) {
  if (n <= 0 || m <= 0) return hipSuccess;
  dim3 grid((unsigned)((m + 3) / 4), n);
  hipLaunchKernelGGL(gather_kernel, grid, dim3(256), 0, s, nodes, m, idx, d);
  return hipGetLastError();
}

hipError_t launch_entry_normalize(const EntryNode* nodes, int n, int64_t m, int, hipStream_t s) {
  if (n <= 0 || m <= 0) return hipSuccess;
  dim3 grid((unsigned)((m + 3) / 4), n);
  hipLaunchKernelGGL(normalize_kernel, grid, dim3(256), 0, s, nodes, m);
  return hipGetLastError();
}

hipError_t launch_entry_finish(const double* vals, const int32_t* expo, int64_t m, long long scale, double* out,
                               hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(finish_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, vals, expo, m, scale, out);
  return hipGetLastError();
}

}  // namespace ht
