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

// In-place Cholesky G = R^T R of the K x K matrix in L (upper triangle used),
// right-looking in the LDL^T form: rows stay unscaled during the elimination
// (one barrier per step) and are divided by sqrt(pivot) at the end.
// sweep 1: pivots <= tol are replaced by tol; sweep 2: such rows are dropped
// (set to zero, dropped[j] = 1).  Returns true if anything was dropped.
__device__ bool chol_lds(double* L, int K, int ld, double tol, int sweep, int* dropped, double* piv) {
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  __shared__ int any;
  if (tid == 0) any = 0;
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    double pj = L[j * ld + j];
    bool drop = false;
    if (!(pj > tol)) {
      if (sweep == 1) pj = tol; else drop = true;
    }
    if (tid == 0) { piv[j] = drop ? 0.0 : pj; dropped[j] = drop ? 1 : 0; if (drop) any = 1; }
    if (!drop) {
      const double inv = 1.0 / pj;
      // row j is read-only during this step: keep this thread's columns of it
      // in registers so the loads and stores of the update can overlap
      double lj[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = j + 1 + tx + 16 * q;
        lj[q] = c < K ? L[j * ld + c] : 0.0;
      }
      for (int a = j + 1 + ty; a < K; a += 16) {
        const double la = L[j * ld + a] * inv;
        double* row = &L[a * ld];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int c = j + 1 + tx + 16 * q;
          if (c < K && c >= a) row[c] -= la * lj[q];
        }
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < K * K; idx += NT) {
    const int a = idx / K, c = idx % K;
    double& v = L[a * ld + c];
    if (c < a || dropped[a]) v = 0.0;
    else {
      const double r = sqrt(piv[a]);
      v = c == a ? r : v / r;
    }
  }
  __syncthreads();
  return any != 0;
}

// In-place inverse of the upper-triangular matrix in L; rows marked in
// `dropped` are treated as having a unit diagonal.  Column j of the inverse is
// -X[0:j,0:j] R[0:j,j] / R[j,j]; each row's dot product is split over 16 lanes
// and reduced with shuffles.
__device__ void trinv_lds(double* L, int K, int ld, const int* dropped, double* y) {
  const int tid = threadIdx.x;
  const int g = tid >> 4, lane = tid & 15;
  for (int j = 0; j < K; ++j) {
    if (tid < j) y[tid] = L[tid * ld + j];
    __syncthreads();
    const double djj = dropped[j] ? 1.0 : L[j * ld + j];
    const double ajj = 1.0 / djj;
    for (int i = g; i < j; i += 16) {
      double x = 0.0;
      for (int k = i + lane; k < j; k += 16) x += L[i * ld + k] * y[k];
      x += __shfl_xor(x, 8, 16);
      x += __shfl_xor(x, 4, 16);
      x += __shfl_xor(x, 2, 16);
      x += __shfl_xor(x, 1, 16);
      if (lane == 0) L[i * ld + j] = -x * ajj;
    }
    if (tid == 0) L[j * ld + j] = ajj;
    __syncthreads();
  }
}

// sweep 1: G -> R1, Ri1 = R1^{-1}.  sweep 2: G2 -> R2 (rows of vanishing
// pivots dropped), R2i = inverse of R2 with unit diagonal on dropped rows.
__global__ __launch_bounds__(NT) void chol_kernel(const SmallArgs* __restrict__ args, int sweep,
                                                  GlobalState* st) {
  __shared__ double L[KMAX * (KMAX + 1)];
  __shared__ double red[NT];
  __shared__ double y[KMAX];
  __shared__ double piv[KMAX];
  __shared__ int dropped[KMAX];
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K, ld = K + 1;
  const int tid = threadIdx.x;
  const double* Gin = sweep == 1 ? a.G : a.G2;
  for (int i = tid; i < K * K; i += NT) L[(i / K) * ld + i % K] = Gin[i];
  for (int i = tid; i < K; i += NT) dropped[i] = 0;
  __syncthreads();
  double md = 0.0;
  bool bad = false;
  for (int i = tid; i < K; i += NT) {
    const double v = L[i * ld + i];
    if (!isfinite(v)) bad = true; else md = fmax(md, v);
  }
  for (int i = tid; i < K * K; i += NT) if (!isfinite(Gin[i])) bad = true;
  const double maxd = block_max(md, red);
  const double badany = block_max(bad ? 1.0 : 0.0, red);
  if (badany > 0.0 && tid == 0) atomicOr(&st->flags, 2u);
  const double tol = maxd > 0.0 ? a.tol_rel * maxd : 1.0;
  const bool ev = chol_lds(L, K, ld, tol, sweep, dropped, piv);
  double* Rout = sweep == 1 ? a.R1 : a.R2;
  double* Riout = sweep == 1 ? a.Ri1 : a.R2i;
  for (int i = tid; i < K * K; i += NT) Rout[i] = L[(i / K) * ld + i % K];
  __syncthreads();
  trinv_lds(L, K, ld, dropped, y);
  for (int i = tid; i < K * K; i += NT) Riout[i] = L[(i / K) * ld + i % K];
  if (sweep == 2 && ev && tid == 0) atomicOr(&st->flags, 1u);
}

// R (= R2 R1, formed by a GEMM) is divided by 2^e, e the binary exponent of
// max |R|; e is added to the scale exponent; Rf = R in the forward type.
__global__ __launch_bounds__(NT) void finish_r_kernel(const SmallArgs* __restrict__ args, GlobalState* st) {
  __shared__ double red[NT];
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K;
  const int tid = threadIdx.x;
  double mx = 0.0;
  for (int i = tid; i < K * K; i += NT) mx = fmax(mx, fabs(a.R[i]));
  const int e = exp2_of(block_max(mx, red));
  for (int i = tid; i < K * K; i += NT) {
    const double v = ldexp(a.R[i], -e);
    a.R[i] = v;
    if (a.rf_type == F32) reinterpret_cast<float*>(a.Rf)[i] = (float)v;
    else reinterpret_cast<double*>(a.Rf)[i] = v;
  }
  if (tid == 0 && e != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->log2_scale), (unsigned long long)(long long)e);
}

// ------------------------------------------------------------------ symmetric eigensolver
// Bhat_t Q_t = Q_t Sigma_t^2 (Section 3.3) for one node per workgroup:
//  1. Householder reduction to tridiagonal form T = H^T Bhat H in LDS; the
//     reflectors are kept in the node's scratch;
//  2. implicit QL iterations with Wilkinson shifts on T: one thread runs the
//     chain of plane rotations of a sweep, all threads then apply them to the
//     rows of Z (one LDS read and write per rotation and row, carried in a
//     register);
//  3. back-transformation Q = H Z, one column of Z per thread;
//  4. eigenvalues sorted descending (clipped at 0) with their columns.
// Q is a product of reflectors and rotations, orthogonal to working precision.
__global__ __launch_bounds__(NT) void eig_kernel(const SmallArgs* __restrict__ args, GlobalState* st) {
  __shared__ double L[KMAX * (KMAX + 1)];
  __shared__ double dg[KMAX], eo[KMAX], rc[KMAX], rs[KMAX], vv[KMAX], pp[KMAX];
  __shared__ double red[NT];
  __shared__ int rankpos[KMAX];
  __shared__ int sh_m, sh_lo, sh_iters;
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K, ld = K + 1;
  const int tid = threadIdx.x;
  double* Vs = a.scratch;                 // reflector k: Vs[k*K + i], i < K-k-1
  double* Ts = a.scratch + K * K;         // tau_k

  for (int i = tid; i < K * K; i += NT) L[(i / K) * ld + i % K] = a.Bh[i];
  __syncthreads();

  // ---- 1. tridiagonalisation: for column k, reflect rows/cols k+1..K-1
  for (int k = 0; k + 2 < K; ++k) {
    const int m = K - k - 1;
    double part = 0.0;
    for (int i = tid; i < m; i += NT) { const double x = L[(k + 1 + i) * ld + k]; part += x * x; }
    const double nrm2 = block_sum(part, red);
    const double x0 = L[(k + 1) * ld + k];
    double tau = 0.0, alpha = x0;
    if (nrm2 > 0.0) {
      alpha = x0 >= 0.0 ? -sqrt(nrm2) : sqrt(nrm2);
      tau = 1.0 / (alpha * (alpha - x0));
    }
    for (int i = tid; i < m; i += NT) vv[i] = i == 0 ? x0 - alpha : L[(k + 1 + i) * ld + k];
    if (tid == 0) { dg[k] = L[k * ld + k]; eo[k] = alpha; Ts[k] = tau; }
    __syncthreads();
    for (int i = tid; i < m; i += NT) Vs[k * K + i] = vv[i];
    if (tau != 0.0) {
      // p = tau A' v over the trailing block A' = L[k+1.., k+1..]
      for (int i = tid; i < m; i += NT) {
        double acc = 0.0;
        const double* row = &L[(k + 1 + i) * ld + k + 1];
        for (int j = 0; j < m; ++j) acc += row[j] * vv[j];
        pp[i] = tau * acc;
      }
      __syncthreads();
      double pv = 0.0;
      for (int i = tid; i < m; i += NT) pv += pp[i] * vv[i];
      const double beta = 0.5 * tau * block_sum(pv, red);
      for (int i = tid; i < m; i += NT) pp[i] -= beta * vv[i];   // w = p - beta v
      __syncthreads();
      // A' <- A' - v w^T - w v^T
      const int ty = tid >> 4, tx = tid & 15;
      for (int i = ty; i < m; i += 16) {
        const double vi = vv[i], wi = pp[i];
        double* row = &L[(k + 1 + i) * ld + k + 1];
        for (int j = tx; j < m; j += 16) row[j] -= vi * pp[j] + wi * vv[j];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (K >= 2) {
      dg[K - 2] = L[(K - 2) * ld + K - 2];
      eo[K - 2] = L[(K - 1) * ld + K - 2];
    }
    dg[K - 1] = L[(K - 1) * ld + K - 1];
    eo[K - 1] = 0.0;
    sh_iters = 0;
  }
  __syncthreads();
  // QL converges at the top of the matrix and keeps the relative accuracy of
  // small eigenvalues only if the tridiagonal grows toward the bottom.
  // Gramians next to the root are graded the other way (large at the top):
  // then T is reversed, T' = P T P, and Z starts as P so that Z = P Z'.
  const bool rev = K > 1 && fabs(dg[0]) > fabs(dg[K - 1]);
  double dtmp = 0.0, etmp = 0.0;
  if (rev) {
    if (tid < K) dtmp = dg[K - 1 - tid];
    if (tid < K - 1) etmp = eo[K - 2 - tid];
  }
  __syncthreads();
  if (rev) {
    if (tid < K) dg[tid] = dtmp;
    if (tid < K - 1) eo[tid] = etmp;
  }
  for (int i = tid; i < K * K; i += NT) {
    const int r = i / K, c = i % K;
    L[r * ld + c] = (rev ? (r + c == K - 1) : (r == c)) ? 1.0 : 0.0;
  }
  __syncthreads();

  // ---- 2. implicit QL on (dg, eo), eo[i] couples i and i+1.  e_m deflates
  // when it is below u (|d_m| + |d_m+1|) or below 1e-18 ||T|| (the rounding
  // level of the Gramian: it moves no eigenvalue by more than that)
  double tloc = 0.0;
  for (int i = tid; i < K; i += NT) tloc = fmax(tloc, fabs(dg[i]) + fabs(eo[i]));
  const double tnorm = block_max(tloc, red);
  const double abs_tol = 1e-18 * tnorm;
  for (int l = 0; l < K; ++l) {
    for (int iter = 0; iter < 80; ++iter) {
      if (tid == 0) sh_m = K - 1;
      __syncthreads();
      for (int m = l + tid; m < K - 1; m += NT) {
        const double e = fabs(eo[m]);
        if (e <= 2.2e-16 * (fabs(dg[m]) + fabs(dg[m + 1])) || e <= abs_tol) atomicMin(&sh_m, m);
      }
      __syncthreads();
      const int m = sh_m;
      __syncthreads();   // every wave has read sh_m before thread 0 may reset it
      if (m == l) break;
      if (tid == 0) {
        double g = (dg[l + 1] - dg[l]) / (2.0 * eo[l]);
        double r = sqrt(g * g + 1.0);
        g = dg[m] - dg[l] + eo[l] / (g + (g >= 0.0 ? r : -r));
        double sn = 1.0, cs = 1.0, p = 0.0;
        double d_i1 = dg[m];                 // dg[i+1] for i = m-1
        double e_i = eo[m - 1], d_i = dg[m - 1];
        int i = m - 1;
        for (; i >= l; --i) {
          // operands of the next rotation, loaded ahead of the dependent chain
          const double e_n = i > l ? eo[i - 1] : 0.0, d_n = i > l ? dg[i - 1] : 0.0;
          const double f = sn * e_i, b = cs * e_i;
          r = sqrt(f * f + g * g);
          eo[i + 1] = r;
          if (r == 0.0) {  // split: restart on the smaller block
            dg[i + 1] = d_i1 - p;
            eo[m] = 0.0;
            break;
          }
          const double ir = 1.0 / r;
          sn = f * ir;
          cs = g * ir;
          g = d_i1 - p;
          r = (d_i - g) * sn + 2.0 * cs * b;
          p = sn * r;
          dg[i + 1] = g + p;
          g = cs * r - b;
          rc[i] = cs;
          rs[i] = sn;
          d_i1 = d_i;
          e_i = e_n;
          d_i = d_n;
        }
        sh_lo = i + 1;   // rotations i = m-1 .. lo were formed
        if (i < l) {
          dg[l] = d_i1 - p;
          eo[l] = g;
          eo[m] = 0.0;
        }
        sh_iters += 1;
      }
      __syncthreads();
      const int lo = sh_lo;
      if (lo <= m - 1) {
        for (int k = tid; k < K; k += NT) {
          double* row = &L[k * ld];
          double carry = row[m];
          for (int i = m - 1; i >= lo; --i) {
            const double x = row[i];
            row[i + 1] = rs[i] * x + rc[i] * carry;
            carry = rc[i] * x - rs[i] * carry;
          }
          row[lo] = carry;
        }
      }
      __syncthreads();
    }
  }

  // ---- 3. Q = H_0 H_1 ... H_{K-3} Z
  for (int k = K - 3; k >= 0; --k) {
    const int m = K - k - 1;
    for (int i = tid; i < m; i += NT) vv[i] = Vs[k * K + i];
    __syncthreads();
    const double tau = Ts[k];
    if (tau != 0.0) {
      for (int j = tid; j < K; j += NT) {
        double y = 0.0;
        for (int i = 0; i < m; ++i) y += vv[i] * L[(k + 1 + i) * ld + j];
        y *= tau;
        for (int i = 0; i < m; ++i) L[(k + 1 + i) * ld + j] -= y * vv[i];
      }
    }
    __syncthreads();
  }

  // ---- 4. sort descending (stable), write Q and lam
  for (int i = tid; i < K; i += NT) {
    const double li = dg[i];
    int pos = 0;
    for (int j = 0; j < K; ++j) {
      const double lj = dg[j];
      if (lj > li || (lj == li && j < i)) ++pos;
    }
    rankpos[i] = pos;
    a.lam[pos] = fmax(li, 0.0);
    if (!isfinite(li)) atomicOr(&st->flags, 2u);
  }
  if (tid == 0) atomicMax(&st->pad, min(sh_iters / K, 255));
  __syncthreads();
  for (int idx = tid; idx < K * K; idx += NT) {
    const int k = idx / K, i = idx % K;
    a.Q[k * K + rankpos[i]] = L[k * ld + i];
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

hipError_t launch_chol(const SmallArgs* args, int n, int sweep, hipStream_t s, GlobalState* st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(chol_kernel, dim3(n), dim3(NT), 0, s, args, sweep, st);
  return hipGetLastError();
}

hipError_t launch_finish_r(const SmallArgs* args, int n, hipStream_t s, GlobalState* st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(finish_r_kernel, dim3(n), dim3(NT), 0, s, args, st);
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
