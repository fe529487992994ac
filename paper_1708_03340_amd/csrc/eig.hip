// Symmetric eigensolver of the reduced Gramians: Bhat_t Q_t = Q_t Sigma_t^2
// (Section 3.3), one workgroup per tree node, the K x K matrix in LDS
// (K <= 128, row stride K + 1).
//  1. Householder reduction to tridiagonal form T = H^T Bhat H; the
//     reflectors are kept in the node's scratch.  Each step's matrix-vector
//     product and rank-2 update load their register tile, compute and store.
//  2. Implicit QL iterations with Wilkinson shifts on T.  One thread runs the
//     chain of plane rotations of a sweep (rotation from one reciprocal square
//     root, operands loaded one rotation ahead); all threads then apply the
//     sweep to the rows of Z, eight columns per LDS round trip.  A tridiagonal
//     that is graded large-at-the-top is reversed first (T' = P T P, Z starts
//     as P): QL keeps the relative accuracy of small eigenvalues only when the
//     matrix grows toward the bottom, and the Gramians next to the root are
//     graded the other way.
//  3. Back-transformation Q = H Z, two threads per column.
//  4. Eigenvalues sorted descending (clipped at 0) with their columns.
// Q is a product of reflectors and rotations, orthogonal to working precision.
#include "dense_util.h"

namespace ht {
namespace {

constexpr int NT = DNT;

__shared__ double g_trash[NT];   // sink for the stores of out-of-range lanes

__global__ __launch_bounds__(NT) void eig_kernel(const SmallArgs* __restrict__ args, GlobalState* st) {
  __shared__ double L[KMAX * (KMAX + 1)];
  __shared__ double dg[KMAX], eo[KMAX], rc[KMAX], rs[KMAX];
  __shared__ double vv[KMAX + 16], pp[KMAX + 16];   // zero beyond the active length
  __shared__ double red[NT / 64];
  __shared__ int rankpos[KMAX];
  __shared__ int sh_m, sh_lo, sh_iters;
  const SmallArgs& a = args[blockIdx.x];
  const int K = a.K, ld = K + 1;
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  double* Vs = a.scratch;                 // reflector k: Vs[k*K + i], i < K-k-1
  double* Ts = a.scratch + K * K;         // tau_k

  for (int i = tid; i < K * K; i += NT) L[(i / K) * ld + i % K] = a.Bh[i];
  __syncthreads();

  // ---- 1. tridiagonalisation
  for (int k = 0; k + 2 < K; ++k) {
    const int m = K - k - 1;
    const double xi = tid < m ? L[(k + 1 + tid) * ld + k] : 0.0;
    const double nrm2 = wg_sum(xi * xi, red);
    const double x0 = L[(k + 1) * ld + k];
    double tau = 0.0, alpha = x0;
    if (nrm2 > 0.0) {
      alpha = x0 >= 0.0 ? -sqrt(nrm2) : sqrt(nrm2);
      tau = 1.0 / (alpha * (alpha - x0));
    }
    if (tid < KMAX + 16) {
      const double v = tid == 0 ? x0 - alpha : xi;   // xi = 0 beyond m
      vv[tid] = v;
      pp[tid] = 0.0;
      if (tid < m) Vs[k * K + tid] = v;
    }
    if (tid == 0) { dg[k] = L[k * ld + k]; eo[k] = alpha; Ts[k] = tau; }
    __syncthreads();
    if (tau != 0.0) {
      double* A = &L[(k + 1) * ld + k + 1];   // trailing block, order m
      // p = tau A v, two threads per row; loads go to clamped addresses
      // (vv is zero past m) so none of them sits behind a branch
      {
        const int r = tid >> 1, h = tid & 1;
        const double* row = &A[min(r, m - 1) * ld];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int c0 = 0; c0 < 64; c0 += 4) {
          if (c0 < m) {
            const int c = h * 64 + c0;
            s0 += row[min(c, m - 1)] * vv[c];
            s1 += row[min(c + 1, m - 1)] * vv[c + 1];
            s2 += row[min(c + 2, m - 1)] * vv[c + 2];
            s3 += row[min(c + 3, m - 1)] * vv[c + 3];
          }
        }
        double sum = (s0 + s1) + (s2 + s3);
        sum += __shfl_xor(sum, 1, 64);
        if (r < m && h == 0) pp[r] = tau * sum;
      }
      __syncthreads();
      const double pv = tid < m ? pp[tid] * vv[tid] : 0.0;
      const double beta = 0.5 * tau * wg_sum(pv, red);
      if (tid < m) pp[tid] -= beta * vv[tid];   // w = p - beta v (zero past m)
      __syncthreads();
      // A <- A - v w^T - w v^T; thread (ty, tx) owns rows ty + 16i and
      // columns tx + 16q, blocks outside the order-m block skipped uniformly
      double va[8], wa[8], vc[8], wc[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        va[i] = vv[ty + 16 * i];
        wa[i] = pp[ty + 16 * i];
        vc[i] = vv[tx + 16 * i];
        wc[i] = pp[tx + 16 * i];
      }
      // all loads first, then all stores (out-of-range lanes store to a
      // trash slot, so no store sits behind a branch)
      double t[8][8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double* rowc = &A[min(ty + 16 * i, m - 1) * ld];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (16 * i < m && 16 * q < m) t[i][q] = rowc[min(tx + 16 * q, m - 1)];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = ty + 16 * i;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int c = tx + 16 * q;
          if (16 * i < m && 16 * q < m)
            *((r < m && c < m) ? &A[r * ld + c] : &g_trash[tid]) = t[i][q] - va[i] * wc[q] - wa[i] * vc[q];
        }
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
  // below u (|d_m| + |d_m+1|) or below 1e-18 ||T|| (the rounding level of the
  // Gramian, which moves no eigenvalue by more than that)
  double tloc = 0.0;
  for (int i = tid; i < K; i += NT) tloc = fmax(tloc, fabs(dg[i]) + fabs(eo[i]));
  const double tnorm = wg_max(tloc, red);
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
      const int m = __builtin_amdgcn_readfirstlane(sh_m);
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
          // operands of the next rotation (unused after the last one)
          const double e_n = eo[max(i - 1, l)], d_n = dg[max(i - 1, l)];
          const double f = sn * e_i, b = cs * e_i;
          const double x2 = f * f + g * g;
          if (x2 == 0.0) {  // split: restart on the smaller block
            eo[i + 1] = 0.0;
            dg[i + 1] = d_i1 - p;
            eo[m] = 0.0;
            break;
          }
          const double ir = rsqrt_nr(x2);
          eo[i + 1] = x2 * ir;
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
      const int lo = __builtin_amdgcn_readfirstlane(sh_lo);
      if (lo <= m - 1) {
        // rotations m-1 .. lo applied to each row of Z, eight per LDS round
        // trip; loads are clamped to lo and invalid lanes of a chunk keep
        // the carry unchanged
        for (int kr = tid; kr < K; kr += NT) {
          double* row = &L[kr * ld];
          double carry = row[m];
          for (int i = m - 1; i >= lo; i -= 8) {
            double xv[8], cv[8], sv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int iu = max(i - u, lo);
              xv[u] = row[iu];
              cv[u] = rc[iu];
              sv[u] = rs[iu];
            }
            double o[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              o[u] = sv[u] * xv[u] + cv[u] * carry;
              const double nc = cv[u] * xv[u] - sv[u] * carry;
              carry = i - u >= lo ? nc : carry;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) *(i - u >= lo ? &row[i - u + 1] : &g_trash[tid]) = o[u];
          }
          row[lo] = carry;
        }
      }
      __syncthreads();
    }
  }

  // ---- 3. Q = H_0 H_1 ... H_{K-3} Z, two threads per column taking the
  // even and odd rows of the reflector; vv is zero past m
  for (int k = K - 3; k >= 0; --k) {
    const int m = K - k - 1;
    if (tid < KMAX + 16) vv[tid] = tid < m ? Vs[k * K + tid] : 0.0;
    __syncthreads();
    const double tau = Ts[k];
    if (tau != 0.0) {
      const int j = tid >> 1, h = tid & 1;
      if (j < K) {
        double* Z = &L[(k + 1) * ld + j];
        double y = 0.0;
        for (int i = h; i < m; i += 16) {
          double zv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) zv[u] = Z[min(i + 2 * u, m - 1) * ld];
#pragma unroll
          for (int u = 0; u < 8; ++u) y += vv[i + 2 * u] * zv[u];
        }
        y += __shfl_xor(y, 1, 64);
        y *= tau;
        for (int i = h; i < m; i += 16) {
          double zv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) zv[u] = Z[min(i + 2 * u, m - 1) * ld];
#pragma unroll
          for (int u = 0; u < 8; ++u)
            *(i + 2 * u < m ? &Z[(i + 2 * u) * ld] : &g_trash[tid]) = zv[u] - y * vv[i + 2 * u];
        }
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

}  // namespace

hipError_t launch_eig(const SmallArgs* args, int n, double*, hipStream_t s, GlobalState* st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(eig_kernel, dim3(n), dim3(NT), 0, s, args, st);
  return hipGetLastError();
}

}  // namespace ht
