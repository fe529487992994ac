// Cholesky steps of CholeskyQR2, one workgroup per tree node, the node's
// K x K Gram matrix resident in LDS (K <= 128, row stride K + 1 so that column
// accesses hit different banks).
//
// Section 3.4 asks for a reduced QR of every leaf frame and of M_{2,3}(B_t);
// CholeskyQR2 gets R from two Gram matrices: G = W^T W = R1^T R1, then
// G2 = (W R1^{-1})^T (W R1^{-1}) = R2^T R2 and R = R2 R1.
//  * sweep 1 clamps pivots that fall below tol (a Gram matrix formed in
//    float32 may be indefinite); the second sweep repairs R;
//  * sweep 2 drops the rows whose pivot vanishes (rank-deficient frames such
//    as those of the sum A + A) and flags them.
// The factor and the inverse are both formed with the matrix held in
// registers across all steps, so a step costs a few LDS reads and at most one
// barrier instead of a round trip of the trailing matrix through LDS.
#include "dense_util.h"

namespace ht {
namespace {

constexpr int NT = DNT;


// Thread (ty, tx) = (tid / 16, tid % 16) owns the entries (ty + 16i, tx + 16q)
// of the upper block triangle q >= i of a KMAX x KMAX matrix: 36 values kept
// in registers for the whole factorisation.
//
// Cholesky G = R^T R, right-looking in LDL^T form (rows stay unscaled and are
// divided by sqrt(pivot) at the end).  Step j reads the pivot row j from a
// double-buffered row in LDS, applies the rank-1 update to the whole register
// tile and the owners of row j+1 publish it (to the row buffer and to L): one
// barrier per step.  Entries of rows or columns that are already eliminated,
// or that lie past K or below the diagonal, receive meaningless updates; they
// never feed an entry that is still live and are never read.
// sweep 1: a pivot <= tol is replaced by tol; sweep 2: its row is dropped
// (dropped[j] = 1, zero row).  Returns true if a row was dropped.  On return
// L holds the scaled R (zero below the diagonal and on dropped rows).
__device__ bool chol_regs(double* L, int K, int ld, double tol, int sweep, int* dropped, double* piv,
                          double (*rowbuf)[KMAX]) {
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  __shared__ int any;
  double v[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int q = i; q < 8; ++q) {
      const int a = ty + 16 * i, c = tx + 16 * q;
      v[i][q] = (a < K && c < K) ? L[a * ld + c] : 0.0;
    }
  if (tid == 0) any = 0;
  if (ty == 0) {   // publish row 0
#pragma unroll
    for (int q = 0; q < 8; ++q) rowbuf[0][tx + 16 * q] = v[0][q];
  }
  for (int j = 0; j < K; ++j) {
    __syncthreads();
    const double* rb = rowbuf[j & 1];
    double pj = rb[j];
    bool drop = false;
    if (!(pj > tol)) {
      if (sweep == 1) pj = tol; else drop = true;
    }
    if (tid == 0) { piv[j] = drop ? 0.0 : pj; dropped[j] = drop ? 1 : 0; if (drop) any = 1; }
    if (!drop) {
      const double inv = rcp_nr(pj);
      double lr[8], lc[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        lr[i] = rb[ty + 16 * i] * inv;
        lc[i] = rb[tx + 16 * i];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = i; q < 8; ++q) v[i][q] -= lr[i] * lc[q];
    }
    // publish row j+1 (after this step's update) into the other buffer and L
    const int jn = j + 1;
    if (jn < K && ty == (jn & 15)) {
      const int ib = jn >> 4;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i == ib) {
#pragma unroll
          for (int q = i; q < 8; ++q) {
            const int c = tx + 16 * q;
            rowbuf[jn & 1][c] = v[i][q];
            if (c < K) L[jn * ld + c] = v[i][q];
          }
        }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < K * K; idx += NT) {
    const int a = idx / K, c = idx % K;
    double& x = L[a * ld + c];
    if (c < a || dropped[a]) x = 0.0;
    else {
      const double r = sqrt(piv[a]);
      x = c == a ? r : x / r;
    }
  }
  __syncthreads();
  return any != 0;
}

// X = R^{-1} for the upper-triangular R in L (rows marked in `dropped` get a
// unit diagonal), column by column: X[i][j] = -(sum_k X[i][k] R[k][j]) / R[j][j]
// for i < j.  Thread (g, l) = (tid / 16, tid % 16) keeps X[g + 16m][l + 16p],
// p >= m, in registers; entries not yet computed are zero, so the dot product
// over its columns needs no masks.  The 16 lanes of a row group (one DPP row)
// sum with DPP moves and the owner of column j stores the result: no
// barriers.  X is written to Xout (K x K, row-major).
__device__ void trinv_regs(const double* L, int K, int ld, const int* dropped, double* Xout) {
  const int tid = threadIdx.x;
  const int g = tid >> 4, l = tid & 15;
  double x[8][8];
#pragma unroll
  for (int m = 0; m < 8; ++m)
#pragma unroll
    for (int p = m; p < 8; ++p) x[m][p] = 0.0;
  for (int j = 0; j < K; ++j) {
    const int jb = j >> 4;
    const double ajj = rcp_nr(dropped[j] ? 1.0 : L[j * ld + j]);
    double r[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) r[p] = L[min(l + 16 * p, K - 1) * ld + j];
    const bool owner = l == (j & 15);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (m <= jb) {     // rows g + 16m < j exist only in blocks m <= j / 16
        double s = 0.0;
#pragma unroll
        for (int p = m; p < 8; ++p)
          if (p <= jb) s += x[m][p] * r[p];
        s = row16_sum(s);
        const int i = g + 16 * m;
        const double xij = i < j ? -s * ajj : (i == j ? ajj : 0.0);
#pragma unroll
        for (int p = m; p < 8; ++p)
          if (p == jb && owner) x[m][p] = xij;
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 8; ++m)
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int i = g + 16 * m, k = l + 16 * p;
      if (i < K && k < K) gst(&Xout[i * K + k], p >= m ? x[m][p] : 0.0);
    }
}

// sweep 1: G -> R1, Ri1 = R1^{-1}.  sweep 2: G2 -> R2 (rows of vanishing
// pivots dropped), R2i = inverse of R2 with unit diagonal on dropped rows.
__global__ __launch_bounds__(NT) void chol_kernel(const SmallArgs* __restrict__ args, int sweep,
                                                  GlobalState* st) {
  __shared__ double L[KMAX * (KMAX + 1)];
  __shared__ double rowbuf[2][KMAX];
  __shared__ double red[NT / 64];
  __shared__ double piv[KMAX];
  __shared__ int dropped[KMAX];
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K, ld = K + 1;
  const int tid = threadIdx.x;
  const double* Gin = sweep == 1 ? a.G : a.G2;
  bool bad = false;
  for (int i = tid; i < K * K; i += NT) {
    const double v = gld(&Gin[i]);
    if (!isfinite(v)) bad = true;
    L[(i / K) * ld + i % K] = v;
  }
  for (int i = tid; i < K; i += NT) dropped[i] = 0;
  __syncthreads();
  double md = 0.0;
  for (int i = tid; i < K; i += NT) {
    const double v = L[i * ld + i];
    if (isfinite(v)) md = fmax(md, v);
  }
  const double maxd = wg_max(md, red);
  const double badany = wg_max(bad ? 1.0 : 0.0, red);
  if (badany > 0.0 && tid == 0) atomicOr(&st->flags, 2u);
  const double tol = maxd > 0.0 ? a.tol_rel * maxd : 1.0;
  const bool ev = chol_regs(L, K, ld, tol, sweep, dropped, piv, rowbuf);
  double* Rout = sweep == 1 ? a.R1 : a.R2;
  double* Riout = sweep == 1 ? a.Ri1 : a.R2i;
  for (int i = tid; i < K * K; i += NT) gst(&Rout[i], L[(i / K) * ld + i % K]);
  trinv_regs(L, K, ld, dropped, Riout);
  if (sweep == 2 && ev && tid == 0) atomicOr(&st->flags, 1u);
}

// R (= R2 R1, formed by a GEMM) is divided by 2^e, e the binary exponent of
// max |R|; e is added to the scale exponent; Rf = R in the forward type.
__global__ __launch_bounds__(NT) void finish_r_kernel(const SmallArgs* __restrict__ args, GlobalState* st) {
  __shared__ double red[NT / 64];
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K;
  const int tid = threadIdx.x;
  double mx = 0.0;
  for (int i = tid; i < K * K; i += NT) mx = fmax(mx, fabs(a.R[i]));
  const int e = exp2_of(wg_max(mx, red));
  for (int i = tid; i < K * K; i += NT) {
    const double v = ldexp(a.R[i], -e);
    a.R[i] = v;
    if (a.rf_type == F32) reinterpret_cast<float*>(a.Rf)[i] = (float)v;
    else reinterpret_cast<double*>(a.Rf)[i] = v;
  }
  if (tid == 0 && e != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->log2_scale), (unsigned long long)(long long)e);
}

}  // namespace

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

}  // namespace ht
