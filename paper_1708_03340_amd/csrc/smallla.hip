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
// One workgroup per tensor: its nodes are args[a0 .. a0 + na) (all nodes of
// the tensor, or a group of them).
__global__ void rank_kernel(const SmallArgs* __restrict__ all_args, const StateRec* __restrict__ recs) {
  __shared__ double red[NT / 64];
  __shared__ int idx_t1, idx_t2;
  const StateRec& R = recs[blockIdx.x];
  const SmallArgs* args = all_args + R.a0;
  const int n = R.na, d = R.d, mode = R.mode, t1 = R.t1, t2 = R.t2;
  const double eps = R.eps;
  GlobalState* st = R.st;
  const int tid = threadIdx.x;
  // ||A||^2 in Gramian units: trace of Bhat_t1 = sum of its eigenvalues
  if (tid == 0) { idx_t1 = -1; idx_t2 = -1; }
  __syncthreads();
  for (int i = tid; i < n; i += NT) {
    if (args[i].node == t1) idx_t1 = i;
    if (args[i].node == t2) idx_t2 = i;
  }
  __syncthreads();
  // a group of nodes without the sons of the root (decomposed later) uses
  // the norm and threshold the group with them stored
  const bool has_root_sons = idx_t1 >= 0;
  double part = 0.0;
  if (has_root_sons)
    for (int i = tid; i < args[idx_t1].K; i += NT) part += args[idx_t1].lam[i];
  const double n2 = wg_sum(part, red);
  double thr;
  if (!has_root_sons) {
    thr = st->thr;
  } else if (R.rel) {
    thr = eps * eps * n2 / (double)(2 * d - 3);
  } else {
    const long long g = st->e_D + st->log2_scale;
    const double en = ldexp(eps, (int)(-g));
    thr = en * en / (double)(2 * d - 3);
  }
  if (tid == 0 && has_root_sons) { st->norm2_units = n2; st->thr = thr; }
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
// forward-product type; optional sigma / ||A||.  Workgroup (node, y) takes
// rows 16y .. 16y + 15 of Q: each thread issues its eight loads together
// (clamped addresses, masked values), stores Qm row-major, and the slab is
// transposed through LDS so that QmT is stored 16 contiguous entries at a
// time.
__global__ void proj_prep_kernel(const SmallArgs* __restrict__ args, const GlobalState* st) {
  __shared__ double tile[16][KMAX + 1];
  const SmallArgs& a = args[blockIdx.x];
  if (a.st) st = a.st;
  const int K = a.K, rc = a.rcap;
  const int r = *a.rank_dev;
  const int i0 = 16 * blockIdx.y;
  const int tid = threadIdx.x;
  if (i0 < K && rc > 0) {
    const int c = tid & 127, ty = tid >> 7;   // 256 threads: two rows per pass
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + ty + 2 * u;
      const double x = a.Q[min(i, K - 1) * K + min(c, K - 1)];
      v[u] = (i < K && c < rc && c < r) ? x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + ty + 2 * u;
      if (a.Qm && i < K && c < rc) a.Qm[i * rc + c] = v[u];
      tile[ty + 2 * u][c] = v[u];
    }
    __syncthreads();
    if (a.QmT) {
      const int ii = tid & 15, c0 = tid >> 4;   // 16 columns per pass
      const int i = i0 + ii;
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        const int cc = c0 + 16 * w;
        if (cc < rc && i < K) {
          const double x = tile[ii][cc];
          if (a.rf_type == F32) reinterpret_cast<float*>(a.QmT)[cc * K + i] = (float)x;
          else reinterpret_cast<double*>(a.QmT)[cc * K + i] = x;
        }
      }
    }
  }
  if (a.sigma_out && blockIdx.y == 0) {
    const double n2 = st->norm2_units;
    for (int i = tid; i < KMAX; i += blockDim.x)
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
// Zero fills, copies and the state kernels take one record per region or
// tensor: blockIdx.y (fills, copies) or the global thread index (state).
__global__ void fill_kernel(const FillRec* __restrict__ recs) {
  const FillRec& r = recs[blockIdx.y];
  uint32_t* p = reinterpret_cast<uint32_t*>(r.p);
  const size_t n = r.bytes / 4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void set_state_kernel(const StateRec* __restrict__ recs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  GlobalState* st = recs[i].st;
  st->log2_scale = recs[i].scale0;
  st->flags = 0;
  st->pad = 0;
  st->alpha_gram = 1.0;
  st->e_D = 0;
  st->norm2_units = 0.0;
  st->thr = 0.0;
  st->alpha_root = 1.0;
}

__global__ void root_norm_kernel(const StateRec* __restrict__ recs) {
  __shared__ double red[NT / 64];
  const StateRec& R = recs[blockIdx.x];
  const double* BD = R.BD;
  const int nel = R.K1 * R.K2;
  double s = 0.0;
  bool bad = false;
  for (int i = threadIdx.x; i < nel; i += NT) {
    const double v = BD[i];
    if (!isfinite(v)) bad = true;
    s += v * v;
  }
  const double tot = wg_sum(s, red);
  const double b = wg_max(bad ? 1.0 : 0.0, red);
  if (threadIdx.x == 0) {
    const int e = exp2_of(sqrt(tot));
    R.st->e_D = e;
    R.st->alpha_gram = ldexp(1.0, -2 * e);
    R.st->alpha_root = ldexp(1.0, -e);
    if (b > 0.0) atomicOr(&R.st->flags, 2u);
  }
}

// One workgroup per record (see PhiRec).
__global__ void phi_scale_kernel(const PhiRec* __restrict__ recs) {
  __shared__ double red[NT / 64];
  const PhiRec& R = recs[blockIdx.x];
  double mx = 0.0, ss = 0.0;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < R.n; i += NT) {
    const double v = R.P[i];
    if (!isfinite(v)) bad = true;
    mx = fmax(mx, fabs(v));
    ss = fma(v, v, ss);
  }
  const double m = wg_max(mx, red);
  const double b = wg_max(bad ? 1.0 : 0.0, red);
  if (R.mode == 2) {
    const double tot = wg_sum(ss, red);
    if (threadIdx.x == 0) {
      const double v = sqrt(tot);
      const int e = exp2_of(v);
      *R.out_val = ldexp(v, -e);
      *R.out_log2 = e + R.add + (R.add_dev ? *R.add_dev : 0);
      if (b > 0.0 && R.flags) atomicOr(R.flags, 2u);
    }
    return;
  }
  const int e = exp2_of(m);
  const double sc = ldexp(1.0, -e);
  for (int64_t i = threadIdx.x; i < R.n; i += NT) R.P[i] *= sc;
  if (threadIdx.x == 0) {
    const long long E = e + (R.E1 ? *R.E1 : 0) + (R.E2 ? *R.E2 : 0);
    if (R.E) *R.E = E;
    if (R.mode == 1) {
      *R.out_val = R.P[0];   // P is 1 x 1, scaled above by this thread
      *R.out_log2 = E + R.add + (R.add_dev ? *R.add_dev : 0);
    }
    if (b > 0.0 && R.flags) atomicOr(R.flags, 2u);
  }
}

__device__ __forceinline__ double ld_any(const void* p, int t, int64_t i) {
  return t == F64 ? reinterpret_cast<const double*>(p)[i] : (double)reinterpret_cast<const float*>(p)[i];
}

// F = H (x) B, F[(p,i), (q,j), (r,l)] = H[p,q,r] B[i,j,l] with the H index
// slowest in every mode.  One record per blockIdx.y; a workgroup takes one
// mode-1 index a = (p,i) at a time, its waves the rows b = (q,j) in turn
// (the pair advanced by additions, no division per row), and the lanes of a
// wave R*L contiguous elements of a row, split into (r, l) by a float
// reciprocal with an exact integer correction (c < 2^24).
__global__ __launch_bounds__(256) void kron_kernel(const KronRec* __restrict__ recs) {
  const KronRec& R = recs[blockIdx.y];
  const int I = R.I, J = R.J, L = R.L, Q = R.Q, RR = R.R;
  const int QJ = Q * J, RL = RR * L;
  const int nA = R.P * I;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nw = blockDim.x >> 6;
  const float invL = 1.0f / (float)L;
  for (int a = blockIdx.x; a < nA; a += gridDim.x) {
    const int p = a / I, i = a - p * I;
    int q = wave / J, j = wave - q * J;
    for (int b = wave; b < QJ; b += nw) {
      const int64_t hb = ((int64_t)p * Q + q) * RR, bb = ((int64_t)i * J + j) * L;
      const int64_t fb = ((int64_t)a * QJ + b) * RL;
      for (int c = lane; c < RL; c += 64) {
        int r = (int)((float)c * invL);
        int l = c - r * L;
        if (l < 0) { --r; l += L; } else if (l >= L) { ++r; l -= L; }
        const double v = ld_any(R.H, R.tH, hb + r) * ld_any(R.B, R.tB, bb + l);
        if (R.tF == F64) reinterpret_cast<double*>(R.F)[fb + c] = v;
        else reinterpret_cast<float*>(R.F)[fb + c] = (float)v;
      }
      j += nw;
      while (j >= J) { j -= J; ++q; }
    }
  }
}

__global__ void write_scale_kernel(const StateRec* __restrict__ recs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const StateRec& R = recs[i];
  const GlobalState* st = R.st;
  if (R.out_scale) *R.out_scale = st->log2_scale + (R.add_eD ? st->e_D : 0);
  if (R.flags) *R.flags = st->flags | ((unsigned)min(st->pad, 255) << 8);
  if (R.root_rank) *R.root_rank = 1;
}

__global__ void copy3_kernel(const CopyRec* __restrict__ recs) {
  const CopyRec& R = recs[blockIdx.y];
  const int64_t n1 = R.n1, n2 = R.n2;
  const int64_t n = R.n0 * n1 * n2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = i / (n1 * n2), r = (i / n2) % n1, c = i % n2;
    const int64_t so = a * R.s0 + r * R.s1 + c * R.s2, dof = a * R.d0 + r * R.d1 + c * R.d2;
    const double v = R.alpha * (R.tsrc == F64 ? reinterpret_cast<const double*>(R.src)[so]
                                              : (double)reinterpret_cast<const float*>(R.src)[so]);
    if (R.tdst == F64) reinterpret_cast<double*>(R.dst)[dof] = v;
    else reinterpret_cast<float*>(R.dst)[dof] = (float)v;
  }
}

constexpr int kMaxY = 65535;   // records per launch along blockIdx.y

}  // namespace

hipError_t launch_fill(const FillRec* r, int n, size_t max_bytes, hipStream_t s) {
  const size_t m = max_bytes / 4;
  if (n <= 0 || m == 0) return hipSuccess;
  const int bx = (int)std::min<size_t>((m + 255) / 256, 4096);
  for (int i0 = 0; i0 < n; i0 += kMaxY) {
    const int ny = std::min(kMaxY, n - i0);
    hipLaunchKernelGGL(fill_kernel, dim3(bx, ny), dim3(256), 0, s, r + i0);
  }
  return hipGetLastError();
}

hipError_t launch_set_state(const StateRec* r, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(set_state_kernel, dim3((n + 63) / 64), dim3(64), 0, s, r, n);
  return hipGetLastError();
}

hipError_t launch_rank_select(const SmallArgs* args, const StateRec* r, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_kernel, dim3(n), dim3(NT), 0, s, args, r);
  return hipGetLastError();
}

hipError_t launch_proj_prep(const SmallArgs* args, int n, const GlobalState* st, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(proj_prep_kernel, dim3(n, KMAX / 16), dim3(256), 0, s, args, st);
  return hipGetLastError();
}

hipError_t launch_sigma_from_lam(const SmallArgs* args, int n, double* const* sig, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sigma_kernel, dim3(n), dim3(128), 0, s, args, sig);
  return hipGetLastError();
}

hipError_t launch_root_norm(const StateRec* r, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(root_norm_kernel, dim3(n), dim3(NT), 0, s, r);
  return hipGetLastError();
}

hipError_t launch_phi_scale(const PhiRec* r, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(phi_scale_kernel, dim3(n), dim3(NT), 0, s, r);
  return hipGetLastError();
}

hipError_t launch_kron(const KronRec* r, int n, int64_t max_elems, int64_t max_a, hipStream_t s) {
  if (n <= 0 || max_elems <= 0 || max_a <= 0) return hipSuccess;
  const int bx = (int)std::min<int64_t>(max_a, 4096);   // one mode-1 index (p, i) per workgroup
  for (int i0 = 0; i0 < n; i0 += kMaxY) {
    const int ny = std::min(kMaxY, n - i0);
    hipLaunchKernelGGL(kron_kernel, dim3(bx, ny), dim3(256), 0, s, r + i0);
  }
  return hipGetLastError();
}

hipError_t launch_write_scale(const StateRec* r, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(write_scale_kernel, dim3((n + 63) / 64), dim3(64), 0, s, r, n);
  return hipGetLastError();
}

hipError_t launch_copy3(const CopyRec* r, int n, int64_t max_elems, hipStream_t s) {
  if (n <= 0 || max_elems <= 0) return hipSuccess;
  const int bx = (int)std::min<int64_t>((max_elems + 255) / 256, 4096);
  for (int i0 = 0; i0 < n; i0 += kMaxY) {
    const int ny = std::min(kMaxY, n - i0);
    hipLaunchKernelGGL(copy3_kernel, dim3(bx, ny), dim3(256), 0, s, r + i0);
  }
  return hipGetLastError();
}

}  // namespace ht
