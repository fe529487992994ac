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
// Every elimination step loads its part of the trailing matrix into
// registers, updates it and stores it back, so one LDS round trip is paid
// per step instead of one per element.
#include "dense_util.h"

namespace ht {
namespace {

constexpr int NT = DNT;

__shared__ double g_trash[NT];   // sink for the stores of out-of-range lanes

// In-place Cholesky G = R^T R (upper triangle) in LDL^T form: rows stay
// unscaled during the elimination and are divided by sqrt(pivot) at the end.
// Thread (ty, tx) owns rows ty + 16i and columns tx + 16q of the trailing
// block; 16 x 16 blocks wholly outside it or below its diagonal are skipped
// on uniform conditions.  Loads use clamped in-range addresses without
// guards (a guarded load compiles to a branch that waits for it); stores of
// out-of-range lanes go to a per-thread trash slot instead of sitting behind a
// branch, which would make every store wait for the previous one.
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
    const int n = K - j - 1;                 // trailing order
    if (!drop && n > 0) {
      const double inv = 1.0 / pj;
      const double* rj = &L[j * ld + j + 1];
      double* T = &L[(j + 1) * ld + j + 1];
      double lr[8], lc[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        lr[i] = rj[min(ty + 16 * i, n - 1)] * inv;
        lc[i] = rj[min(tx + 16 * i, n - 1)];
      }
      // all loads of the step first, then all stores: the compiler cannot
      // move a load above a store to the same array by itself
      double v[8][8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int ac = min(ty + 16 * i, n - 1);
#pragma unroll
        for (int q = i; q < 8; ++q)
          if (16 * q < n) v[i][q] = T[ac * ld + min(tx + 16 * q, n - 1)];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int a = ty + 16 * i;
#pragma unroll
        for (int q = i; q < 8; ++q) {
          if (16 * q < n) {
            const int c = tx + 16 * q;
            const bool ok = a < n && c < n && c >= a;
            *(ok ? &T[a * ld + c] : &g_trash[tid]) = v[i][q] - lr[i] * lc[q];
          }
        }
      }
    }
    __syncthreads();
  }
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

// In-place inverse of the upper-triangular matrix in L (rows marked in
// `dropped` get a unit diagonal).  Column j of the inverse is
// -X[0:j, 0:j] R[0:j, j] / R[j, j] with X the part already inverted; each row's
// dot product is split over 16 lanes and reduced with shuffles.  y holds
// column j of R zero-padded to KMAX, so the products need no guards.
__device__ void trinv_lds(double* L, int K, int ld, const int* dropped, double* y) {
  const int tid = threadIdx.x;
  const int g = tid >> 4, lane = tid & 15;
  for (int j = 0; j < K; ++j) {
    if (tid < KMAX) y[tid] = tid < j ? L[min(tid, K - 1) * ld + j] : 0.0;
    __syncthreads();
    const double djj = dropped[j] ? 1.0 : L[j * ld + j];
    const double ajj = 1.0 / djj;
    double yk[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) yk[p] = y[lane + 16 * p];
    double x[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      x[m] = 0.0;
      if (16 * m < j) {
        const double* row = &L[min(g + 16 * m, K - 1) * ld];
#pragma unroll
        for (int p = 0; p < 8; ++p)
          if (16 * p < j) x[m] += row[min(lane + 16 * p, K - 1)] * yk[p];
      }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (16 * m < j) {
        double s = x[m];
        s += __shfl_xor(s, 8, 16);
        s += __shfl_xor(s, 4, 16);
        s += __shfl_xor(s, 2, 16);
        s += __shfl_xor(s, 1, 16);
        const int i = g + 16 * m;
        *((lane == 0 && i < j) ? &L[i * ld + j] : &g_trash[tid]) = -s * ajj;
      }
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
  __shared__ double red[NT / 64];
  __shared__ double y[KMAX];
  __shared__ double piv[KMAX];
  __shared__ int dropped[KMAX];
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K, ld = K + 1;
  const int tid = threadIdx.x;
  const double* Gin = sweep == 1 ? a.G : a.G2;
  bool bad = false;
  for (int i = tid; i < K * K; i += NT) {
    const double v = Gin[i];
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
