// Symmetric eigensolver of the reduced Gramians: Bhat_t Q_t = Q_t Sigma_t^2
// (Section 3.3), one workgroup of 256 threads per tree node, K <= 128.
//
//  1. Householder reduction to tridiagonal form T = H^T Bhat H with the matrix
//     in registers (thread (ty, tx) holds rows ty + 16i, columns tx + 16q).
//     A step publishes column k through LDS, forms p = tau A v with DPP sums
//     along the 16 lanes of a row group, and applies the rank-2 update in
//     registers: three barriers per step.  The reflectors go to the node's
//     scratch.
//  2. Implicit QL iterations with Wilkinson shifts on T, pipelined: wave 0
//     finds the next unreduced block and runs the chain of plane rotations of
//     the next sweep (one lane; rotation from a reciprocal square root refined
//     by one third-order step), while waves 1-3 apply the previous sweep to
//     the rows of Z in LDS.  One barrier per sweep.  A tridiagonal graded
//     large-at-the-top is reversed first (T' = P T P, Z starts as P): QL keeps
//     the relative accuracy of small eigenvalues only when the matrix grows
//     toward the bottom, and the Gramians next to the root are graded the
//     other way.
//  3. Back-transformation Q = H_0 ... H_{K-3} Z with Z in registers, the 16
//     lanes of a DPP row holding the rows of a column strip: no barriers.
//  4. Eigenvalues sorted descending (clipped at 0) with their columns.
// Q is a product of reflectors and rotations, orthogonal to working precision.
#include "dense_util.h"

namespace ht {
namespace {

constexpr int NT = DNT;

// 1 / sqrt(x), x > 0 normal: hardware estimate (relative error ~5e-8) and one
// third-order step, y (1 + e/2 + 3e^2/8) with e = 1 - x y^2.
__device__ __forceinline__ double rsqrt3(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

// Sum over a wave of 64 lanes, returned to every lane: DPP sums in rows of
// 16, then the four row sums.
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  return ((lane_val(v, 0) + lane_val(v, 16)) + lane_val(v, 32)) + lane_val(v, 48);
}

enum : int { SWEEP_NONE = 0, SWEEP_ROT = 1, SWEEP_DONE = 2 };

// KT: the largest order the instantiation takes (64, 96 or 128).  Up to 96 a
// node's LDS is at most 80 KB and two nodes share a CU (the registers of the
// rotation blocks keep it from more).
template <int KT>
__global__ __launch_bounds__(NT, KT <= 96 ? 2 : 1) void eig_kernel(const SmallArgs* __restrict__ args,
                                                                   GlobalState* st) {
  constexpr int RB = KT / 16;                    // row (column) blocks of 16
  __shared__ double L[KT * (KT + 1)];            // Z during the QL phase (column K: store sink)
  __shared__ double dg[KT], eo[KT];
  // the vectors of the tridiagonalisation and, later, the rotations of two
  // QL sweeps share one buffer
  __shared__ double vbuf[4 * KT];
  double* const xs = vbuf;
  double* const ps = vbuf + KT;
  double (*const rcs)[KT] = reinterpret_cast<double (*)[KT]>(vbuf);
  double (*const rss)[KT] = reinterpret_cast<double (*)[KT]>(vbuf + 2 * KT);
  __shared__ int sw_state[2], sw_m[2], sw_lo[2];
  __shared__ double part[16];
  __shared__ int rankpos[KT];
  const SmallArgs& a = args[blockIdx.x];
  if (a.st) st = a.st;
  const int K = a.K, ld = K + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ty = tid >> 4, tx = tid & 15;
  double* Vs = a.scratch;                 // reflector k: Vs[k*K + i], i < K-k-1
  double* Ts = a.scratch + K * K;         // tau_k

  // ---- 1. tridiagonalisation, A in registers
  {
    double A[RB][RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int r = ty + 16 * i, c = tx + 16 * q;
        A[i][q] = (r < K && c < K) ? gld(&a.Bh[r * K + c]) : 0.0;
      }
    for (int k = 0; k + 2 < K; ++k) {
      const int kb = k >> 4;
      // publish column k below the diagonal, and the diagonal entry
      if (tx == (k & 15)) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
          if (q == kb) {
#pragma unroll
            for (int i = 0; i < RB; ++i) {
              const int r = ty + 16 * i;
              xs[r] = r > k ? A[i][q] : 0.0;
              if (r == k) dg[k] = A[i][q];
            }
          }
      }
      __syncthreads();
      // every wave forms ||x||^2 itself (the same sum in the same order)
      const double x0 = xs[k + 1];
      double hi = 0.0;   // entries 64 .. KT-1 (lanes past KT-64 add zero)
      if (KT > 64) hi = xs[min(lane + 64, KT - 1)] * (lane + 64 < KT ? 1.0 : 0.0);
      const double nrm2 = wave_sum(xs[lane] * xs[lane] + hi * hi);
      double tau = 0.0, alpha = x0;
      if (nrm2 > 0.0) {
        alpha = x0 >= 0.0 ? -sqrt(nrm2) : sqrt(nrm2);
        tau = 1.0 / (alpha * (alpha - x0));
      }
      if (tid == 0) { eo[k] = alpha; gst(&Ts[k], tau); }
      if (tid > k && tid < K) gst(&Vs[k * K + tid - k - 1], tid == k + 1 ? x0 - alpha : xs[tid]);
      if (tau != 0.0) {
        // v (zero at indices <= k) at this thread's rows and columns
        double vr[RB], vc[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          const int r = ty + 16 * i, c = tx + 16 * i;
          vr[i] = r == k + 1 ? x0 - alpha : xs[r];
          vc[i] = c == k + 1 ? x0 - alpha : xs[c];
        }
        // p = tau A v at this thread's rows, summed over the 16 lanes of the row group
        double pr[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          double s = 0.0;
#pragma unroll
          for (int q = 0; q < RB; ++q) s = fma(A[i][q], vc[q], s);
          pr[i] = tau * row16_sum(s);
        }
        // v . p: partial over the 8 rows of the group, joined across groups in LDS
        double vp = 0.0;
#pragma unroll
        for (int i = 0; i < RB; ++i) vp = fma(vr[i], pr[i], vp);
        if (tx == 0) {
          part[ty] = vp;
#pragma unroll
          for (int i = 0; i < RB; ++i) ps[ty + 16 * i] = pr[i];
        }
        __syncthreads();
        double tot = 0.0;
#pragma unroll
        for (int g = 0; g < 16; ++g) tot += part[g];
        const double beta = 0.5 * tau * tot;
        double wr[RB], wc[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          const int r = ty + 16 * i, c = tx + 16 * i;
          wr[i] = r > k ? pr[i] - beta * vr[i] : 0.0;
          wc[i] = c > k ? ps[c] - beta * vc[i] : 0.0;
        }
        // A <- A - v w^T - w v^T (entries with an index <= k are unchanged)
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int q = 0; q < RB; ++q) A[i][q] -= vr[i] * wc[q] + wr[i] * vc[q];
      }
      __syncthreads();   // xs, ps, part are reused by the next step
    }
    // the trailing 2 x 2 (or smaller) block
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int r = ty + 16 * i, c = tx + 16 * q;
        if (K >= 2 && r == K - 2 && c == K - 2) dg[K - 2] = A[i][q];
        if (K >= 2 && r == K - 1 && c == K - 2) eo[K - 2] = A[i][q];
        if (r == K - 1 && c == K - 1) dg[K - 1] = A[i][q];
      }
    if (tid == 0) {
      eo[K - 1] = 0.0;
      sw_state[0] = sw_state[1] = SWEEP_NONE;
    }
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
  if (wave == 0)
    for (int i = lane; i < K; i += 64) tloc = fmax(tloc, fabs(dg[i]) + fabs(eo[i]));
  for (int off = 32; off > 0; off >>= 1) tloc = fmax(tloc, __shfl_xor(tloc, off, 64));
  const double abs_tol = 1e-18 * tloc;   // used by wave 0 only
  int l = 0, iter = 0;                   // producer state (wave 0)
  int max_it = 0;                        // most sweeps any one eigenvalue took (wave 0)
  bool noconv = false;                   // an eigenvalue was given up on (wave 0)
  // Finds the next sweep and writes its rotations into buffer b (wave 0 only).
  auto produce = [&](int b) {
    while (true) {
      if (l >= K) {
        if (lane == 0) sw_state[b] = SWEEP_DONE;
        return;
      }
      int m = K - 1;
      for (int base = l; base < K - 1; base += 64) {
        const int idx = base + lane;
        bool neg = false;
        if (idx < K - 1) {
          const double e = fabs(eo[idx]);
          neg = e <= 2.2e-16 * (fabs(dg[idx]) + fabs(dg[idx + 1])) || e <= abs_tol;
        }
        const unsigned long long bal = __ballot(neg);
        if (bal) {
          m = base + __ffsll((long long)bal) - 1;
          break;
        }
      }
      if (m == l || iter >= 80) {   // converged (or given up on): next eigenvalue
        max_it = max(max_it, iter);
        if (m != l) noconv = true;   // 80 sweeps without e[l] reaching the deflation test
        ++l;
        iter = 0;
        continue;
      }
      ++iter;
      if (lane == 0) {
        double g = (dg[l + 1] - dg[l]) / (2.0 * eo[l]);
        double r = sqrt(g * g + 1.0);
        g = dg[m] - dg[l] + eo[l] / (g + (g >= 0.0 ? r : -r));
        double sn = 1.0, cs = 1.0, p = 0.0;
        double d_i1 = dg[m];                 // d[i+1] for i = m-1
        // rotations i = m-1 .. l.  Whole blocks of eight run as straight-line
        // code: their operands (e[i], d[i]) are loaded one block ahead and
        // their results (e[i+1], d[i+1], c_i, s_i) stored after the block, so
        // neither an LDS access nor a branch sits on the dependent chain.  A
        // block in which a rotation meets f = g = 0 (a split) is redone
        // rotation by rotation, as is the tail of fewer than eight.
        int lo = l;
        bool split = false;
        // one rotation with the split test; false on a split at index i
        auto step = [&](int i, double e_i, double d_i) -> bool {
          const double f = sn * e_i, bb = cs * e_i;
          const double x2 = f * f + g * g;
          if (x2 == 0.0) {  // split: restart on the smaller block
            eo[i + 1] = 0.0;
            dg[i + 1] = d_i1 - p;
            lo = i + 1;
            return false;
          }
          const double ir = rsqrt3(x2);
          eo[i + 1] = x2 * ir;
          sn = f * ir;
          cs = g * ir;
          g = d_i1 - p;
          r = (d_i - g) * sn + 2.0 * cs * bb;
          p = sn * r;
          dg[i + 1] = g + p;
          g = cs * r - bb;
          rcs[b][i] = cs;
          rss[b][i] = sn;
          d_i1 = d_i;
          return true;
        };
        // Rotation u of a block consumes the operands (eb[u], db[u]) and at
        // once loads those of rotation u of the next block into the same
        // registers, so the loop carries no copies.  A block that meets
        // x2 = 0 ends with g and p not finite (the reciprocal square root of
        // zero turns every later quantity into NaN); it is redone rotation by
        // rotation from its operands in LDS, unchanged until its results are
        // stored.
        double eb[8], db[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int idx = max(m - 1 - u, l);
          eb[u] = eo[idx];
          db[u] = dg[idx];
        }
        int i0 = m - 1;
        while (i0 - 7 >= l) {
          const double sn0 = sn, cs0 = cs, p0 = p, g0 = g, d0 = d_i1;
          double oe[8], od[8], oc[8], os[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const double f = sn * eb[u], bb = cs * eb[u];
            const double x2 = f * f + g * g;
            const double ir = rsqrt3(x2);
            oe[u] = x2 * ir;
            sn = f * ir;
            cs = g * ir;
            g = d_i1 - p;
            r = (db[u] - g) * sn + 2.0 * cs * bb;
            p = sn * r;
            od[u] = g + p;
            g = cs * r - bb;
            oc[u] = cs;
            os[u] = sn;
            d_i1 = db[u];
            const int idx = max(i0 - 8 - u, l);
            eb[u] = eo[idx];
            db[u] = dg[idx];
          }
          if (isfinite(g) && isfinite(p)) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int i = i0 - u;
              eo[i + 1] = oe[u];
              dg[i + 1] = od[u];
              rcs[b][i] = oc[u];
              rss[b][i] = os[u];
            }
          } else {   // redo the block rotation by rotation
            sn = sn0; cs = cs0; p = p0; g = g0; d_i1 = d0;
            for (int u = 0; u < 8 && !split; ++u) split = !step(i0 - u, eo[i0 - u], dg[i0 - u]);
            if (split) break;
          }
          i0 -= 8;
        }
        // the tail: fewer than eight rotations, operands already in eb, db
        for (int u = 0; u < 8 && !split && i0 - u >= l; ++u) split = !step(i0 - u, eb[u], db[u]);
        if (split) {
          eo[m] = 0.0;
        } else {
          dg[l] = d_i1 - p;
          eo[l] = g;
          eo[m] = 0.0;
        }
        sw_m[b] = m;
        sw_lo[b] = lo;   // rotations m-1 .. lo were formed
        sw_state[b] = SWEEP_ROT;
      }
      return;
    }
  };
  if (wave == 0) produce(0);
  __syncthreads();
  for (int b = 0;; b ^= 1) {
    if (sw_state[b] == SWEEP_DONE) break;
    if (wave == 0) {
      produce(b ^ 1);
    } else {
      // apply sweep b: rotations m-1 .. lo to each row of Z, eight per LDS
      // round trip; loads are clamped to lo and invalid lanes keep the carry
      const int m = sw_m[b], lo = sw_lo[b];
      const double* rc = rcs[b];
      const double* rs = rss[b];
      const int kr = tid - 64;
      if (kr < K && lo <= m - 1) {
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
          for (int u = 0; u < 8; ++u) *(i - u >= lo ? &row[i - u + 1] : &row[K]) = o[u];
        }
        row[lo] = carry;
      }
    }
    __syncthreads();
  }

  // ---- 3. Q = H_0 H_1 ... H_{K-3} Z with Z in registers: thread (cg, rl) =
  // (tid / 16, tid % 16) holds Z[rl + 16i][cg + 16q]; a DPP row is one column strip
  const int rl = tid & 15, cg = tid >> 4;
  double Z[RB][RB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int r = rl + 16 * i, c = cg + 16 * q;
      Z[i][q] = (r < K && c < K) ? L[r * ld + c] : 0.0;
    }
  if (K >= 3) {
    double vn[RB];
    double taun = 0.0;
    auto load_v = [&](int k) {
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int r = rl + 16 * i;
        vn[i] = (r > k && r < K) ? gld(&Vs[k * K + r - k - 1]) : 0.0;
      }
      taun = gld(&Ts[k]);
    };
    load_v(K - 3);
    for (int k = K - 3; k >= 0; --k) {
      double v[RB];
#pragma unroll
      for (int i = 0; i < RB; ++i) v[i] = vn[i];
      const double tau = taun;
      if (k > 0) load_v(k - 1);   // next reflector, in flight during this one
      if (tau != 0.0) {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          double s = 0.0;
#pragma unroll
          for (int i = 0; i < RB; ++i) s = fma(v[i], Z[i][q], s);
          const double y = tau * row16_sum(s);
#pragma unroll
          for (int i = 0; i < RB; ++i) Z[i][q] = fma(-v[i], y, Z[i][q]);
        }
      }
    }
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
    gst(&a.lam[pos], fmax(li, 0.0));
    if (!isfinite(li)) atomicOr(&st->flags, 2u);
  }
  if (tid == 0) {   // wave 0, lane 0: the producer's counters
    atomicMax(&st->pad, min(max_it, 255));
    if (noconv) atomicOr(&st->flags, 8u);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int r = rl + 16 * i, c = cg + 16 * q;
      if (r < K && c < K) gst(&a.Q[r * K + rankpos[c]], Z[i][q]);
    }
}

}  // namespace

hipError_t launch_eig(const SmallArgs* args, int n, int max_k, hipStream_t s, GlobalState* st) {
  if (n <= 0) return hipSuccess;
  if (max_k <= 64)
    hipLaunchKernelGGL(eig_kernel<64>, dim3(n), dim3(NT), 0, s, args, st);
  else if (max_k <= 96)
    hipLaunchKernelGGL(eig_kernel<96>, dim3(n), dim3(NT), 0, s, args, st);
  else
    hipLaunchKernelGGL(eig_kernel<128>, dim3(n), dim3(NT), 0, s, args, st);
  return hipGetLastError();
}

}  // namespace ht
