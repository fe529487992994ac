// Small dense float64 kernels of the truncation, one workgroup per tree node,
// the node's K x K matrix resident in LDS (K <= 128, 128 KiB of the 160 KiB).
//
//  * chol_kernel      -- the two Cholesky steps of CholeskyQR2 (Section 3.4 asks
//                        for a reduced QR of every leaf frame and of every
//                        M_{2,3}(B_t); CholeskyQR2 gets R from Gram matrices):
//                        sweep 1 clamps vanishing pivots, sweep 2 drops the
//                        directions whose pivot vanishes (rank-deficient
//                        frames such as the sum A + A), forms R = R2 R1 and
//                        R^{-1}, divides R by a power of two and records it.
//  * eig_kernel       -- cyclic Jacobi eigensolver of the reduced Gramians
//                        (Bhat_t Q_t = Q_t Sigma_t^2, Section 3.3), parallel
//                        circle ordering, eigenvalues in descending order.
//  * rank_select      -- fixed ranks or the tolerance rule.
//  * proj_prep        -- masked leading eigenvectors for the projections.
#include "ht_internal.h"

namespace ht {
namespace {

constexpr int NT = 256;

__device__ double block_max(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int exp2_of(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 0;
  int e;
  frexp(x, &e);
  return e;
}

// In-place Cholesky G = R^T R of the K x K matrix in L (upper triangle used).
// sweep 1: pivots <= tol are replaced by tol; sweep 2: such rows are dropped
// (set to zero, dropped[j] = 1).  Returns true if anything was dropped/clamped.
__device__ bool chol_lds(double* L, int K, double tol, int sweep, int* dropped) {
  const int tid = threadIdx.x;
  __shared__ int any;
  if (tid == 0) any = 0;
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    double piv = L[j * K + j];
    bool drop = false;
    if (!(piv > tol)) {
      if (sweep == 1) piv = tol; else drop = true;
    }
    __syncthreads();
    if (drop) {
      for (int c = j + tid; c < K; c += NT) L[j * K + c] = 0.0;
      if (tid == 0) { dropped[j] = 1; any = 1; }
    } else {
      const double r = sqrt(piv);
      const double inv = 1.0 / r;
      for (int c = j + 1 + tid; c < K; c += NT) L[j * K + c] *= inv;
      if (tid == 0) { L[j * K + j] = r; dropped[j] = 0; }
      __syncthreads();
      const int nrem = K - j - 1;
      for (int idx = tid; idx < nrem * nrem; idx += NT) {
        const int a = j + 1 + idx / nrem, c = j + 1 + idx % nrem;
        if (c >= a) L[a * K + c] -= L[j * K + a] * L[j * K + c];
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < K * K; idx += NT) {
    const int a = idx / K, c = idx % K;
    if (c < a) L[idx] = 0.0;
  }
  __syncthreads();
  return any != 0;
}

// In-place inverse of the upper-triangular matrix in L; rows marked in
// `dropped` are treated as having a unit diagonal.
__device__ void trinv_lds(double* L, int K, const int* dropped, double* y) {
  const int tid = threadIdx.x;
  for (int j = 0; j < K; ++j) {
    if (tid < j) y[tid] = L[tid * K + j];
    __syncthreads();
    const double djj = dropped[j] ? 1.0 : L[j * K + j];
    const double ajj = 1.0 / djj;
    if (tid < j) {
      double x = 0.0;
      for (int k = tid; k < j; ++k) x += L[tid * K + k] * y[k];
      L[tid * K + j] = -x * ajj;
    }
    if (tid == 0) L[j * K + j] = ajj;
    __syncthreads();
  }
}

__global__ __launch_bounds__(NT) void chol_kernel(const SmallArgs* __restrict__ args, int sweep,
                                                  GlobalState* st) {
  __shared__ double L[KMAX * KMAX];
  __shared__ double red[NT];
  __shared__ double y[KMAX];
  __shared__ int dropped[KMAX];
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K;
  const int tid = threadIdx.x;
  const double* Gin = sweep == 1 ? a.G : a.G2;
  for (int i = tid; i < K * K; i += NT) L[i] = Gin[i];
  for (int i = tid; i < K; i += NT) dropped[i] = 0;
  __syncthreads();
  double md = 0.0;
  bool bad = false;
  for (int i = tid; i < K; i += NT) {
    const double v = L[i * K + i];
    if (!isfinite(v)) bad = true; else md = fmax(md, v);
  }
  for (int i = tid; i < K * K; i += NT) if (!isfinite(L[i])) bad = true;
  const double maxd = block_max(md, red);
  const double badany = block_max(bad ? 1.0 : 0.0, red);
  if (badany > 0.0 && tid == 0) atomicOr(&st->flags, 2u);
  const double tol = maxd > 0.0 ? a.tol_rel * maxd : 1.0;
  const bool ev = chol_lds(L, K, tol, sweep, dropped);

  if (sweep == 1) {
    for (int i = tid; i < K * K; i += NT) a.R1[i] = L[i];
    __syncthreads();
    trinv_lds(L, K, dropped, y);
    for (int i = tid; i < K * K; i += NT) a.Ri1[i] = L[i];
    return;
  }
  if (ev && tid == 0) atomicOr(&st->flags, 1u);
  // R = R2 R1 (both upper triangular), written unnormalised first
  double mx = 0.0;
  for (int idx = tid; idx < K * K; idx += NT) {
    const int i = idx / K, c = idx % K;
    double v = 0.0;
    if (c >= i)
      for (int k = i; k <= c; ++k) v += L[i * K + k] * a.R1[k * K + c];
    a.R[idx] = v;
    mx = fmax(mx, fabs(v));
  }
  const double gmx = block_max(mx, red);
  const int e = exp2_of(gmx);
  __syncthreads();
  for (int idx = tid; idx < K * K; idx += NT) {
    const double v = ldexp(a.R[idx], -e);
    a.R[idx] = v;
    if (a.rf_type == F32) reinterpret_cast<float*>(a.Rf)[idx] = (float)v;
    else reinterpret_cast<double*>(a.Rf)[idx] = v;
  }
  // Ri = R1^{-1} R2^{-1}
  trinv_lds(L, K, dropped, y);
  for (int idx = tid; idx < K * K; idx += NT) {
    const int i = idx / K, c = idx % K;
    double v = 0.0;
    if (c >= i)
      for (int k = i; k <= c; ++k) v += a.Ri1[i * K + k] * L[k * K + c];
    a.Ri[idx] = v;
  }
  if (tid == 0 && e != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->log2_scale), (unsigned long long)(long long)e);
}

// ------------------------------------------------------------------ Jacobi eigensolver
// Circle (round-robin) ordering: Ke = K rounded up to even, Ke-1 rounds of
// Ke/2 disjoint pairs; index >= K is a dummy.
__device__ __forceinline__ int circle_pos(int i, int r, int Ke) {
  return i == 0 ? 0 : 1 + ((i - 1 + r) % (Ke - 1));
}

__global__ __launch_bounds__(NT) void eig_kernel(const SmallArgs* __restrict__ args, GlobalState* st) {
  __shared__ double L[KMAX * KMAX];
  __shared__ double cs_c[KMAX / 2], cs_s[KMAX / 2];
  __shared__ int pp[KMAX / 2], qq[KMAX / 2];
  __shared__ double red[NT];
  __shared__ int nrot;
  __shared__ int rankpos[KMAX];
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K;
  const int tid = threadIdx.x;
  const int Ke = K + (K & 1);
  const int npair = Ke / 2, nround = Ke - 1;
  double* Ag = a.scratch;                 // A while V is in LDS
  double* Vg = a.scratch + K * K;         // V while A is in LDS
  double* CS = a.scratch + 2 * K * K;     // rotations of one sweep: nround x npair x 2

  for (int i = tid; i < K * K; i += NT) {
    L[i] = a.Bh[i];
    Vg[i] = (i / K == i % K) ? 1.0 : 0.0;
  }
  __syncthreads();
  double fs = 0.0;
  for (int i = tid; i < K * K; i += NT) fs += L[i] * L[i];
  const double normA = sqrt(block_sum(fs, red));
  const double floor_abs = 1e-18 * normA;

  for (int sweep = 0; sweep < 40 && K > 1; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int r = 0; r < nround; ++r) {
      if (tid < npair) {
        int p = circle_pos(tid, r, Ke), q = circle_pos(Ke - 1 - tid, r, Ke);
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < K) {
          const double app = L[p * K + p], aqq = L[q * K + q], apq = L[p * K + q];
          if (fabs(apq) > floor_abs && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            atomicAdd(&nrot, 1);
          }
        } else {
          q = p;  // dummy pair: identity
        }
        pp[tid] = p; qq[tid] = q; cs_c[tid] = c; cs_s[tid] = s;
        CS[(r * npair + tid) * 2] = c;
        CS[(r * npair + tid) * 2 + 1] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int idx = tid; idx < npair * K; idx += NT) {
        const int j = idx / K, k = idx % K;
        const double c = cs_c[j], s = cs_s[j];
        if (s != 0.0) {
          const int p = pp[j], q = qq[j];
          const double x = L[p * K + k], yv = L[q * K + k];
          L[p * K + k] = c * x - s * yv;
          L[q * K + k] = s * x + c * yv;
        }
      }
      __syncthreads();
      // columns: A <- A J
      for (int idx = tid; idx < npair * K; idx += NT) {
        const int k = idx / npair, j = idx % npair;
        const double c = cs_c[j], s = cs_s[j];
        if (s != 0.0) {
          const int p = pp[j], q = qq[j];
          const double x = L[k * K + p], yv = L[k * K + q];
          L[k * K + p] = c * x - s * yv;
          L[k * K + q] = s * x + c * yv;
        }
      }
      __syncthreads();
      if (tid < npair && cs_s[tid] != 0.0) {
        L[pp[tid] * K + qq[tid]] = 0.0;
        L[qq[tid] * K + pp[tid]] = 0.0;
      }
      __syncthreads();
    }
    const int rot = nrot;
    __syncthreads();
    if (rot == 0) break;
    // apply this sweep's rotations to V (V <- V J), V swapped into LDS
    for (int i = tid; i < K * K; i += NT) { Ag[i] = L[i]; L[i] = Vg[i]; }
    __syncthreads();
    for (int r = 0; r < nround; ++r) {
      if (tid < npair) {
        int p = circle_pos(tid, r, Ke), q = circle_pos(Ke - 1 - tid, r, Ke);
        if (p > q) { int t = p; p = q; q = t; }
        if (q >= K) q = p;
        pp[tid] = p; qq[tid] = q;
        cs_c[tid] = CS[(r * npair + tid) * 2];
        cs_s[tid] = CS[(r * npair + tid) * 2 + 1];
      }
      __syncthreads();
      for (int idx = tid; idx < npair * K; idx += NT) {
        const int k = idx / npair, j = idx % npair;
        const double c = cs_c[j], s = cs_s[j];
        if (s != 0.0) {
          const int p = pp[j], q = qq[j];
          const double x = L[k * K + p], yv = L[k * K + q];
          L[k * K + p] = c * x - s * yv;
          L[k * K + q] = s * x + c * yv;
        }
      }
      __syncthreads();
    }
    for (int i = tid; i < K * K; i += NT) { Vg[i] = L[i]; L[i] = Ag[i]; }
    __syncthreads();
  }
  // sort eigenvalues descending (stable), write Q and lam
  for (int i = tid; i < K; i += NT) {
    const double li = L[i * K + i];
    int pos = 0;
    for (int j = 0; j < K; ++j) {
      const double lj = L[j * K + j];
      if (lj > li || (lj == li && j < i)) ++pos;
    }
    rankpos[i] = pos;
    a.lam[pos] = fmax(li, 0.0);
    if (!isfinite(li)) atomicOr(&st->flags, 2u);
  }
  __syncthreads();
  for (int idx = tid; idx < K * K; idx += NT) {
    const int k = idx / K, i = idx % K;
    a.Q[k * K + rankpos[i]] = Vg[k * K + i];
  }
}

// ------------------------------------------------------------------ ranks
__global__ void rank_kernel(const SmallArgs* __restrict__ args, int n, int d, int mode, double eps,
                            int rel, int t1, int t2, GlobalState* st) {
  __shared__ double red[NT];
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
  const double n2 = block_sum(part, red);
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
  __shared__ double red[NT];
  double s = 0.0;
  bool bad = false;
  for (int i = threadIdx.x; i < K1 * K2; i += NT) {
    const double v = BD[i];
    if (!isfinite(v)) bad = true;
    s += v * v;
  }
  const double tot = block_sum(s, red);
  const double b = block_max(bad ? 1.0 : 0.0, red);
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
  if (flags) *flags = st->flags;
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

hipError_t launch_chol(const SmallArgs* args, int n, int sweep, hipStream_t s, GlobalState* st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(chol_kernel, dim3(n), dim3(NT), 0, s, args, sweep, st);
  return hipGetLastError();
}

hipError_t launch_eig(const SmallArgs* args, int n, double*, hipStream_t s, GlobalState* st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(eig_kernel, dim3(n), dim3(NT), 0, s, args, st);
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
