// Small float64 kernels of the truncation around the dense node solvers
// (the Cholesky and eigensolver kernels live in chol.hip and eig.hip):
//  * rank_kernel      -- fixed ranks or the tolerance rule of Section 3.3;
//  * proj_prep_kernel -- masked leading eigenvectors for the projections;
//  * sigma_kernel     -- singular values from the Gramian eigenvalues;
//  * state kernels    -- scale exponent, flags and the root normalisation;
//  * fill / copy      -- zero fills and strided copies with type conversion.
#include "dense_util.h"

namespace ht {
namespace {

constexpr int NT = DNT;


// ------------------------------------------------------------------ ranks
__global__ void rank_kernel(const SmallArgs* __restrict__ args, int n, int d, int mode, double eps,
                            int rel, int t1, int t2, GlobalState* st) {
  __shared__ double red[NT / 64];
  __shared__ int idx_t1, idx_t2;
  const int tid = threadIdx.x;
  // ||A||^2 in Gramian units: trace of Bhat_t1 = sum of its eigenvalues
  if (tid == 0) { idx_t1 = -1; idx_t2 = -1; }
  __syncthreads();
  for (int i = tid; i < n; i += NT) {
    if (args[i].node == t1) idx_t1 = i;
    if (args[i].node == t2) idx_t2 = i;
  }
  __syncthreads();
  double part = 0.0;
  if (idx_t1 >= 0)
    for (int i = tid; i < args[idx_t1].K; i += NT) part += args[idx_t1].lam[i];
  const double n2 = wg_sum(part, red);
  double thr;
  if (rel) {
    thr = eps * eps * n2 / (double)(2 * d - 3);
  } else {
    const long long g = st->e_D + st->log2_scale;
    const double en = ldexp(eps, (int)(-g));
    thr = en * en / (double)(2 * d - 3);
  }
  if (tid == 0) { st->norm2_units = n2; st->thr = thr; }
  for (int i = tid; i < n; i += NT) {
    const SmallArgs& a = args[i];
    int r;
    if (mode == 0) {
      r = a.rfix;
    } else {
      // smallest r >= 1 with sum_{j >= r} lam_j <= thr (0-based tail)
      double tail = 0.0;
      r = a.K;
      for (int j = a.K - 1; j >= 1; --j) {
        tail += a.lam[j];
        if (tail <= thr) r = j; else break;
      }
      if (r < 1) r = 1;
      if (r > a.rcap) {
        r = a.rcap;
        atomicOr(&st->flags, 4u);
      }
    }
    *a.rank_dev = r;
  }
  __syncthreads();
  if (tid == 0 && mode != 0 && idx_t1 >= 0 && idx_t2 >= 0) {
    int r = *args[idx_t1].rank_dev;
    if (r > args[idx_t2].rcap) r = args[idx_t2].rcap;
    *args[idx_t1].rank_dev = r;
    *args[idx_t2].rank_dev = r;
  }
}

// Qm = Q[:, :rcap] with columns >= r zeroed (float64); QmT = Qm^T in the
// forward-product type; optional sigma / ||A||.
__global__ void proj_prep_kernel(const SmallArgs* __restrict__ args, const GlobalState* st) {
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K, rc = a.rcap;
  const int r = *a.rank_dev;
  for (int idx = threadIdx.x; idx < K * rc; idx += blockDim.x) {
    const int i = idx / rc, c = idx % rc;
    const double v = c < r ? a.Q[i * K + c] : 0.0;
    if (a.Qm) a.Qm[idx] = v;
    if (a.QmT) {
      if (a.rf_type == F32) reinterpret_cast<float*>(a.QmT)[c * K + i] = (float)v;
      else reinterpret_cast<double*>(a.QmT)[c * K + i] = v;
    }
  }
  if (a.sigma_out) {
    const double n2 = st->norm2_units;
    for (int i = threadIdx.x; i < KMAX; i += blockDim.x)
      a.sigma_out[i] = (i < K && n2 > 0.0) ? sqrt(a.lam[i] / n2) : 0.0;
  }
}

__global__ void sigma_kernel(const SmallArgs* __restrict__ args, double* const* sig) {
  const SmallArgs& a = args[blockIdx.x];
  double* out = sig[blockIdx.x];
  if (!out) return;
  for (int i = threadIdx.x; i < a.K; i += blockDim.x) out[i] = sqrt(a.lam[i]);
}

// ------------------------------------------------------------------ misc
__global__ void fill_kernel(uint32_t* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void set_state_kernel(GlobalState* st, long long scale0) {
  st->log2_scale = scale0;
  st->flags = 0;
  st->pad = 0;
  st->alpha_gram = 1.0;
  st->e_D = 0;
  st->norm2_units = 0.0;
  st->thr = 0.0;
}

__global__ void root_norm_kernel(const double* BD, int K1, int K2, GlobalState* st) {
  __shared__ double red[NT / 64];
  double s = 0.0;
  bool bad = false;
  for (int i = threadIdx.x; i < K1 * K2; i += NT) {
    const double v = BD[i];
    if (!isfinite(v)) bad = true;
    s += v * v;
  }
  const double tot = wg_sum(s, red);
  const double b = wg_max(bad ? 1.0 : 0.0, red);
  if (threadIdx.x == 0) {
    const int e = exp2_of(sqrt(tot));
    st->e_D = e;
    st->alpha_gram = ldexp(1.0, -2 * e);
    if (b > 0.0) atomicOr(&st->flags, 2u);
  }
}

__global__ void write_scale_kernel(const GlobalState* st, long long* out, unsigned int* flags,
                                   int* root_rank, int add_eD) {
  if (out) *out = st->log2_scale + (add_eD ? st->e_D : 0);
  if (flags) *flags = st->flags | ((unsigned)min(st->pad, 255) << 8);
  if (root_rank) *root_rank = 1;
}

__global__ void copy3_kernel(const void* src, int tsrc, void* dst, int tdst, int64_t n0, int64_t n1,
                             int64_t n2, int64_t s0, int64_t s1, int64_t s2, int64_t d0, int64_t d1,
                             int64_t d2, double alpha) {
  const int64_t n = n0 * n1 * n2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = i / (n1 * n2), r = (i / n2) % n1, c = i % n2;
    const int64_t so = a * s0 + r * s1 + c * s2, dof = a * d0 + r * d1 + c * d2;
    const double v = alpha * (tsrc == F64 ? reinterpret_cast<const double*>(src)[so]
                                          : (double)reinterpret_cast<const float*>(src)[so]);
    if (tdst == F64) reinterpret_cast<double*>(dst)[dof] = v;
    else reinterpret_cast<float*>(dst)[dof] = (float)v;
  }
}

}  // namespace

hipError_t launch_fill(void* ptr, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, s, reinterpret_cast<uint32_t*>(ptr), n);
  return hipGetLastError();
}

hipError_t launch_set_state(GlobalState* st, long long scale0, hipStream_t s) {
  hipLaunchKernelGGL(set_state_kernel, dim3(1), dim3(1), 0, s, st, scale0);
  return hipGetLastError();
}

hipError_t launch_rank_select(const SmallArgs* args, int n, int d, int mode, double eps, int rel,
                              int, int t1, int t2, GlobalState* st, hipStream_t s) {
  hipLaunchKernelGGL(rank_kernel, dim3(1), dim3(NT), 0, s, args, n, d, mode, eps, rel, t1, t2, st);
  return hipGetLastError();
}

hipError_t launch_proj_prep(const SmallArgs* args, int n, const GlobalState* st, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(proj_prep_kernel, dim3(n), dim3(256), 0, s, args, st);
  return hipGetLastError();
}

hipError_t launch_sigma_from_lam(const SmallArgs* args, int n, double* const* sig, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sigma_kernel, dim3(n), dim3(128), 0, s, args, sig);
  return hipGetLastError();
}

hipError_t launch_root_norm(const double* BD, int K1, int K2, GlobalState* st, hipStream_t s) {
  hipLaunchKernelGGL(root_norm_kernel, dim3(1), dim3(NT), 0, s, BD, K1, K2, st);
  return hipGetLastError();
}

hipError_t launch_write_scale(const GlobalState* st, long long* out, unsigned int* flags, int* root_rank,
                              int add_eD, hipStream_t s) {
  hipLaunchKernelGGL(write_scale_kernel, dim3(1), dim3(1), 0, s, st, out, flags, root_rank, add_eD);
  return hipGetLastError();
}

hipError_t launch_copy3(const void* src, int tsrc, void* dst, int tdst, int64_t n0, int64_t n1, int64_t n2,
                        int64_t s0, int64_t s1, int64_t s2, int64_t d0, int64_t d1, int64_t d2, double alpha,
                        hipStream_t s) {
  const int64_t n = n0 * n1 * n2;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(copy3_kernel, dim3(blocks), dim3(256), 0, s, src, tsrc, dst, tdst, n0, n1, n2, s0, s1,
                     s2, d0, d1, d2, alpha);
  return hipGetLastError();
}

}  // namespace ht
