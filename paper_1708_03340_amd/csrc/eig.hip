// Symmetric eigensolver of the reduced Gramians: Bhat_t Q_t = Q_t Sigma_t^2
// (Section 3.3), one workgroup of 256 threads per tree node, K <= 128.
//
//  1. Householder reduction to tridiagonal form T = H^T Bhat H with the matrix
//     in registers (thread (ty, tx) holds rows ty + 16i, columns tx + 16q).
//     A step publishes column k through LDS, forms p = tau A v with DPP sums
//     along the 16 lanes of a row group, and applies the rank-2 update in
//     registers: three barriers per step.  The reflectors go to the node's
//     scratch.
//  2. Divide and conquer on T (Cuppen's tearing), all merges of one depth of
//     the halving tree at once.  T, scaled to max-norm 1, is torn at every
//     row boundary: T = diag(T_1, T_2) + rho v v^T with v = e_m + sign(b) e_m+1,
//     rho = |b|, so the blocks start as single rows d_i - |e_i-1| - |e_i|.  A
//     merge of two blocks with eigen-decompositions Q_j D_j Q_j^T solves the
//     rank-one update D + rho z z^T, z = Q^T v / sqrt(2) (rho doubled):
//       - the eigenvalues are sorted; entries with rho |z_j| below
//         2 u max(max|D| of the block, u), and pairs of poles closer than that
//         after a plane rotation of their z entries, deflate (a wave per merge at
//         the top four depths, else a thread, runs the scan and rotates the
//         two eigenvector columns);
//       - each remaining root of 1 + rho sum_j z_j^2 / (d_j - lambda) = 0 is
//         found by a pair of threads: origin at the nearer pole, a start from the
//         two nearest poles with the other terms frozen at the midpoint, then
//         the two-pole model matching psi, psi' and phi, phi' (Bunch, Nielsen
//         and Sorensen), bracketed by bisection;
//       - z is recomputed from the roots (Gu and Eisenstat), which makes the
//         vectors z_j / (d_j - lambda_i) orthogonal to working precision;
//       - the merged block's eigenvectors are the product of the two blocks'
//         eigenvectors (Z in LDS) with those vectors (written to scratch),
//         eight by eight outputs per thread, columns in ascending order.
//  3. Back-transformation Q = H_0 ... H_{K-3} Z with Z in registers, the 16
//     lanes of a DPP row holding the rows of a column strip: no barriers.
//  4. Eigenvalues sorted descending (clipped at 0) with their columns.
// Q is a product of reflectors, plane rotations and the merge products,
// orthogonal to working precision.
#include "dense_util.h"

namespace ht {
namespace {

constexpr int NT = DNT;

// Sum over a wave of 64 lanes, returned to every lane: DPP sums in rows of
// 16, then the four row sums.
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  return ((lane_val(v, 0) + lane_val(v, 16)) + lane_val(v, 32)) + lane_val(v, 48);
}

constexpr double kUnit = 1.1102230246251565e-16;   // unit roundoff of float64

// Root x in (Alo, Ahi) of c + b1 / (Alo - x) + b2 / (Ahi - x) = 0, where one
// of Alo, Ahi is zero (the origin pole) and b1, b2 > 0.  Mirrored so that the
// origin is the lower pole, then the smaller root of the quadratic in its
// cancellation-free form.  Not finite when the model has no such root.
__device__ __forceinline__ double dc_quad(double c, double b1, double b2, double Alo, double Ahi) {
  const bool low = Alo == 0.0;
  const double cc = low ? c : -c, p1 = low ? b1 : b2, p2 = low ? b2 : b1, W = low ? Ahi : -Alo;
  const double B = -(cc * W + p1 + p2), C = p1 * W;
  const double sq = sqrt(fmax(fma(B, B, -4.0 * cc * C), 0.0));
  const double y = -B >= 0.0 ? 2.0 * C / (-B + sq) : (-B - sq) / (2.0 * cc);
  return low ? y : -y;
}

// The other lane of a pair (2x, 2x+1), by DPP quad_perm [1,0,3,2] (a VALU
// move; both lanes of the pair are active wherever these are used).
__device__ __forceinline__ double pair_other(double v) { return dpp_f64<0xB1>(v); }
__device__ __forceinline__ int pair_other(int v) { return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true); }

// Sum over the two lanes of a pair.
__device__ __forceinline__ double pair_sum(double v) { return v + pair_other(v); }

// Root i of the secular equation 1 + rho sum_j z_j^2 / (d_j - lambda) = 0
// for poles d[0] < ... < d[nk-1] (the root lies in (d_i, d_i+1), the last
// one in (d_nk-1, d_nk-1 + rho |z|^2]), found by the two lanes of a pair, each
// summing every other pole (par = lane parity).  Returns lambda = d[org] + tau
// with the origin pole org and the offset tau (so d_j - lambda is formed as
// (d_j - d_org) - tau, without cancellation).  *iters: iterations taken;
// *conv: false if the iteration limit was reached.
__device__ void dc_root(int i, int nk, const double* d, const double* z, double rho, int par, int* org_out,
                        double* tau_out, int* iters, bool* conv) {
  int org;
  double lo_t, hi_t, tau;
  if (i < nk - 1) {
    const double di = d[i], hw = 0.5 * (d[i + 1] - di);
    double f = 0.0;
    #pragma unroll 4
    for (int j = par; j < nk; j += 2) {
      const double del = (d[j] - di) - hw;
      f += rho * z[j] * z[j] * rcp_nr(del);
    }
    f = 1.0 + pair_sum(f);
    const double wi = rho * z[i] * z[i], wi1 = rho * z[i + 1] * z[i + 1];
    const double ti = wi * rcp_nr(-hw), ti1 = wi1 * rcp_nr((d[i + 1] - di) - hw);
    if (f >= 0.0) {
      org = i; lo_t = 0.0; hi_t = hw; tau = hw;
    } else {
      org = i + 1; lo_t = -hw; hi_t = 0.0; tau = -hw;
    }
    // the two nearest poles with their own weights, the rest frozen
    const double x0 = dc_quad(f - ti - ti1, wi, wi1, d[i] - d[org], d[i + 1] - d[org]);
    if (lo_t < x0 && x0 < hi_t) tau = x0;
  } else {
    double zz = 0.0;
    for (int j = par; j < nk; j += 2) zz += z[j] * z[j];
    zz = pair_sum(zz);
    org = nk - 1; lo_t = 0.0; hi_t = rho * zz; tau = hi_t;
  }
  const double dorg = d[org];
  const double Alo = d[i] - dorg, Ahi = i + 1 < nk ? d[i + 1] - dorg : 0.0;
  int it = 0;
  bool ok = false;
  for (; it < 64; ++it) {
    double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0, sabs = 0.0;
    #pragma unroll 4
    for (int j = par; j < nk; j += 2) {
      const double inv = rcp_nr((d[j] - dorg) - tau);
      const double tj = rho * z[j] * z[j] * inv, dtj = tj * inv;
      if (j <= i) { psi += tj; dpsi += dtj; } else { phi += tj; dphi += dtj; }
      sabs += fabs(tj);
    }
    psi = pair_sum(psi); dpsi = pair_sum(dpsi); phi = pair_sum(phi); dphi = pair_sum(dphi);
    sabs = pair_sum(sabs);
    const double f = 1.0 + psi + phi;
    if (fabs(f) <= kUnit * (8.0 * (1.0 + sabs) + fabs(tau) * (dpsi + dphi))) { ok = true; break; }
    if (f > 0.0) hi_t = tau; else lo_t = tau;
    const double dlo = Alo - tau;
    const double b1 = dpsi * dlo * dlo, a1 = psi - b1 / dlo;
    double x;
    if (i < nk - 1) {
      const double dhi = Ahi - tau;
      const double b2 = dphi * dhi * dhi, a2 = phi - b2 / dhi;
      x = dc_quad(1.0 + a1 + a2, b1, b2, Alo, Ahi);
    } else {
      const double c = 1.0 + a1;
      x = c > 0.0 ? b1 / c : hi_t + 1.0;   // no model root: bisect
    }
    if (!(lo_t < x && x < hi_t)) {
      x = 0.5 * (lo_t + hi_t);
      if (!(lo_t < x && x < hi_t)) { ok = true; break; }   // bracket down to adjacent doubles
    }
    if (x == tau) { ok = true; break; }
    tau = x;
  }
  *org_out = org;
  *tau_out = tau;
  *iters = it;
  *conv = ok;
}

// KT: the largest order the instantiation takes (64, 96 or 128).  Up to 96 a
// node's LDS is at most 80 KB and two nodes share a CU.
template <int KT>
__global__ __launch_bounds__(NT, KT <= 96 ? 2 : 1) void eig_kernel(const SmallArgs* __restrict__ args,
                                                                   GlobalState* st) {
  constexpr int RB = KT / 16;                    // row (column) blocks of 16
  constexpr int PADC = KT > 96 ? 1 : 0;          // row padding of Z (LDS permitting)
  __shared__ double L[KT * (KT + PADC)];         // Z, rows of the tridiagonal basis
  __shared__ double dg[KT], eo[KT];              // diagonal (later: eigenvalues), off-diagonal
  // the vectors of the tridiagonalisation, then four per-position arrays of
  // the merges: sorted eigenvalues (compacted to the kept poles), their z
  // entries, the new eigenvalue of each position, the root offsets
  __shared__ double vbuf[4 * KT];
  double* const xs = vbuf;
  double* const ps = vbuf + KT;
  double* const part = vbuf + 2 * KT;            // 16 partial sums
  double* const ds = vbuf;
  double* const zs = vbuf + KT;
  double* const nv = vbuf + 2 * KT;
  double* const taus = vbuf + 3 * KT;
  __shared__ double zh[KT];                      // recomputed z of the kept poles
  // per position of a merged block: child column in sorted order; kept
  // position of kept index j; kept index of a position (255: deflated);
  // origin pole of root i; new column of a position (later: sort rank)
  __shared__ unsigned char perm[KT], kidx[KT], jof[KT], orgs[KT], newcol[KT];
  __shared__ unsigned char kcnt[64];             // kept poles per merge of a depth
  __shared__ int sh_maxit, sh_noconv;
  const SmallArgs& a = args[blockIdx.x];
  if (a.st) st = a.st;
  const int K = a.K, ld = K + PADC;
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
    // max |A|: a column below the diagonal with norm under u^2 max|A| is
    // taken as zero (no reflection).  Its square may leave the float64
    // range, and alpha (alpha - x0) with it, which would make tau infinite;
    // the entries it drops are below the deflation floor of step 2.
    double thr;
    {
      double m = 0.0;
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int q = 0; q < RB; ++q) m = fmax(m, fabs(A[i][q]));
      for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
      if (lane == 0) part[wave] = m;
      __syncthreads();
      double amax = part[0];
      for (int w = 1; w < NT / 64; ++w) amax = fmax(amax, part[w]);
      const double fl = kUnit * kUnit * amax;
      thr = fl * fl;
      __syncthreads();   // part is reused below
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
      if (nrm2 > thr && nrm2 > 0.0) {
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
      sh_maxit = 0;
      sh_noconv = 0;
    }
  }
  __syncthreads();

  // ---- 2. divide and conquer on (dg, eo); eo[i] couples rows i and i+1
  {
    double amax = 0.0;
    for (int i = tid; i < K; i += NT) amax = fmax(amax, fmax(fabs(dg[i]), fabs(eo[i])));
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) zh[wave] = amax;
    __syncthreads();
    const double scale = fmax(fmax(zh[0], zh[1]), fmax(zh[2], zh[3]));
    // Z = I; single rows d_i - |e_i-1| - |e_i| (all scaled by 1 / scale)
    for (int i = tid; i < K * ld; i += NT) L[i] = (i / ld == i % ld) ? 1.0 : 0.0;
    const bool run = K >= 2 && scale > 0.0 && isfinite(scale);
    const double inv = run ? 1.0 / scale : 1.0;
    if (run && tid < K) {
      const double em = tid > 0 ? fabs(eo[tid - 1]) : 0.0, ep = tid < K - 1 ? fabs(eo[tid]) : 0.0;
      dg[tid] = (dg[tid] * inv - em * inv) - ep * inv;
    }
    __syncthreads();
    if (run && tid < K) eo[tid] *= inv;
    __syncthreads();
    const int T = run ? dc_depths(K) : 0;
    int64_t vbase = eig_reflector_doubles(K);
    double* const scr = a.scratch;
    // two threads per position x of the tridiagonal (K <= 128 = NT / 2)
    const int x = tid >> 1, h = tid & 1;
    for (int t = T - 1; t >= 0; --t) {
      const int M = ((K - 1) >> t) + 1;          // rows of the largest block at this depth
      // the merge of position x: block b of depth t
      int b = 0, lo = 0, mid = 0, hi = 0;
      bool mine = false;
      if (x < K) {
        b = (((x + 1) << t) + K - 1) / K - 1;
        lo = (b * K) >> t;
        hi = ((b + 1) * K) >> t;
        mid = ((2 * b + 1) * K) >> (t + 1);
        mine = lo < mid && mid < hi;
      }
      const int m = hi - lo;
      const double rho = mine ? 2.0 * fabs(eo[mid - 1]) : 0.0;

      // (a) sort the two blocks' eigenvalues; z = Q^T v / sqrt(2)
      if (mine) {
        const double v = dg[x];
        int r = 0;
        for (int y = lo + h; y < hi; y += 2) {
          const double w = dg[y];
          r += (w < v || (w == v && y < x)) ? 1 : 0;
        }
        r += pair_other(r);
        r = min(r, m - 1);
        if (h == 0) {
          const double sgn = eo[mid - 1] >= 0.0 ? 1.0 : -1.0;
          const double zx = (x < mid ? L[(mid - 1) * ld + x] : sgn * L[mid * ld + x]) * 0.70710678118654752;
          perm[lo + r] = (unsigned char)x;
          ds[lo + r] = v;
          zs[lo + r] = zx;
        }
      }
      __syncthreads();

      // (b) deflation: the sorted entries of a merge are scanned in order by
      // a wave (at most four merges at this depth; its lanes rotate the rows
      // of two eigenvector columns) or by a single thread; kept poles are
      // compacted in place
      {
        const bool wide = (1 << t) <= NT / 64;
        const int g = wide ? wave : tid, gl = wide ? lane : 0, gs = wide ? 64 : 1;
        for (int bb = g; bb < (1 << t); bb += wide ? NT / 64 : NT) {
          const int blo = (bb * K) >> t, bhi = ((bb + 1) * K) >> t, bmid = ((2 * bb + 1) * K) >> (t + 1);
          if (!(blo < bmid && bmid < bhi)) continue;
          const int bm = bhi - blo;
          const double brho = 2.0 * fabs(eo[bmid - 1]);
          // block-relative, with an absolute floor of 2 u^2 (T has max-norm 1):
          // eigenvalues below u^2 are far under the float64 resolution of the
          // Gramian, and poles or weights at those scales make the secular
          // equation and the eigenvector entries z_j / (d_j - lambda) overflow
          const double tol = 2.0 * kUnit * fmax(fmax(fabs(ds[blo]), fabs(ds[bhi - 1])), kUnit);
          int nk = 0, pk = -1;
          for (int p = 0; p < bm; ++p) {
            const int P = blo + p;
            const double zp = zs[P], dp = ds[P];
            if (brho * fabs(zp) <= tol) {
              if (gl == 0) { nv[P] = dp; jof[P] = 255; }
              continue;
            }
            if (pk >= 0) {
              const int PK = blo + pk;
              const double zq = zs[PK], dq = ds[PK];
              const double tau = sqrt(fma(zq, zq, zp * zp));
              const double c = zp / tau, sn = -zq / tau;
              if (fabs((dp - dq) * c * sn) <= tol) {
                // rotate so that z_pk = 0: position pk deflates
                const int ca = perm[PK], cb = perm[P];
                for (int r = blo + gl; r < bhi; r += gs) {
                  const double u = L[r * ld + ca], w = L[r * ld + cb];
                  L[r * ld + ca] = c * u + sn * w;
                  L[r * ld + cb] = c * w - sn * u;
                }
                if (gl == 0) {
                  zs[P] = tau;
                  nv[PK] = dq * c * c + dp * sn * sn;
                  jof[PK] = 255;
                  ds[P] = dq * sn * sn + dp * c * c;
                }
              } else {
                if (gl == 0) {
                  kidx[blo + nk] = (unsigned char)pk;
                  jof[PK] = (unsigned char)nk;
                  ds[blo + nk] = dq;
                  zs[blo + nk] = zq;
                }
                ++nk;
              }
            }
            pk = p;
          }
          if (pk >= 0) {
            const int PK = blo + pk;
            const double dq = ds[PK], zq = zs[PK];
            if (gl == 0) {
              kidx[blo + nk] = (unsigned char)pk;
              jof[PK] = (unsigned char)nk;
              ds[blo + nk] = dq;
              zs[blo + nk] = zq;
            }
            ++nk;
          }
          if (gl == 0) kcnt[bb] = (unsigned char)nk;
        }
      }
      __syncthreads();

      // (c) two threads per root of the secular equation
      const int nk = mine ? kcnt[b] : 0;
      const int i = x - lo;
      if (mine && i < nk) {
        int org, its;
        double tau;
        bool conv;
        dc_root(i, nk, ds + lo, zs + lo, rho, h, &org, &tau, &its, &conv);
        if (h == 0) {
          orgs[x] = (unsigned char)org;
          taus[x] = tau;
          nv[lo + kidx[x]] = ds[lo + org] + tau;
          atomicMax(&sh_maxit, its);
          if (!conv) sh_noconv = 1;
        }
      }
      __syncthreads();

      // (d) z recomputed from the roots (kept index j = i); new column of
      // every position: rank of its new eigenvalue in the block
      if (mine) {
        const double* d = ds + lo;
        if (i < nk) {
          const double dj = d[i];
          double w = h == 0 ? (taus[x] - (dj - d[orgs[x]])) / rho : 1.0;   // (lambda_j - d_j) / rho
          #pragma unroll 4
          for (int q = h; q < nk; q += 2) {
            if (q == i) continue;
            const double lq = (d[orgs[lo + q]] - dj) + taus[lo + q];   // lambda_q - d_j
            w *= lq * rcp_nr(d[q] - dj);
          }
          w *= pair_other(w);
          if (h == 0) zh[x] = copysign(sqrt(fmax(w, 0.0)), zs[x]);
        }
        const double v = nv[x];
        int r = 0;
        for (int y = lo + h; y < hi; y += 2) {
          const double u = nv[y];
          r += (u < v || (u == v && y < x)) ? 1 : 0;
        }
        r += pair_other(r);
        if (h == 0) newcol[x] = (unsigned char)min(r, m - 1);
      }
      __syncthreads();

      // (e) column newcol[x] of the merge's m x m vector block V (row p: the
      // sorted position p): e_p for a deflated position, else the normalised
      // root vector zhat_j / (d_j - lambda_i); the two threads of x take
      // alternate rows
      double* const V = scr + vbase + (int64_t)lo * M;
      if (mine) {
        const int c = newcol[x];
        const int ji = jof[x];
        if (ji == 255) {
          for (int p = h; p < m; p += 2) gst(&V[p * m + c], p == i ? 1.0 : 0.0);
        } else {
          const double* d = ds + lo;
          const double lo_org = d[orgs[lo + ji]], tl = taus[lo + ji];
          double ss = 0.0;
          #pragma unroll 4
          for (int q = h; q < nk; q += 2) {
            const double u = zh[lo + q] * rcp_nr((d[q] - lo_org) - tl);
            ss = fma(u, u, ss);
          }
          const double nrm = rsqrt_nr(pair_sum(ss));
          for (int p = h; p < m; p += 2) {
            const int q = jof[lo + p];
            const double u = q == 255 ? 0.0 : zh[lo + q] * rcp_nr((d[q] - lo_org) - tl) * nrm;
            gst(&V[p * m + c], u);
          }
        }
      }
      __threadfence_block();
      __syncthreads();

      // (f) Z[lo:hi, lo:hi] <- Z[lo:hi, perm] V, eight by eight outputs per
      // thread; tiles of all merges of the depth are numbered in order (at
      // most ceil(K/8)^2 <= NT of them for K <= 128)
      double acc[8][8];
      int tr0 = -1, tc0 = 0, tlo = 0, thi = 0;
      {
        int f = tid;
        for (int bb = 0; bb < (1 << t); ++bb) {
          const int blo = (bb * K) >> t, bhi = ((bb + 1) * K) >> t, bmid = ((2 * bb + 1) * K) >> (t + 1);
          if (!(blo < bmid && bmid < bhi)) continue;
          const int nt = (bhi - blo + 7) >> 3;
          if (f < nt * nt) {
            tr0 = blo + 8 * (f / nt);
            tc0 = 8 * (f % nt);
            tlo = blo;
            thi = bhi;
            break;
          }
          f -= nt * nt;
        }
      }
      if (tr0 >= 0) {
        const int bm = thi - tlo;
        const double* Vb = scr + vbase + (int64_t)tlo * M;
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int w = 0; w < 8; ++w) acc[u][w] = 0.0;
        int rows[8], cols[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          rows[u] = min(tr0 + u, thi - 1) * ld;
          cols[u] = min(tc0 + u, bm - 1);
        }
        // the operands of product p + 1 are loaded before the products of p
        double zn[8], vn[8];
        {
          const int col = perm[tlo];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            zn[u] = L[rows[u] + col];
            vn[u] = gld(&Vb[cols[u]]);
          }
        }
        for (int p = 0; p < bm; ++p) {
          double zr[8], vr[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            zr[u] = zn[u];
            vr[u] = vn[u];
          }
          const int pn = min(p + 1, bm - 1);
          const int col = perm[tlo + pn];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            zn[u] = L[rows[u] + col];
            vn[u] = gld(&Vb[pn * bm + cols[u]]);
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int w = 0; w < 8; ++w) acc[u][w] = fma(zr[u], vr[w], acc[u][w]);
        }
      }
      __syncthreads();
      if (tr0 >= 0) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int w = 0; w < 8; ++w)
            if (tr0 + u < thi && tc0 + w < thi - tlo) L[(tr0 + u) * ld + tlo + tc0 + w] = acc[u][w];
      }
      if (mine && h == 0) dg[lo + newcol[x]] = nv[x];
      __syncthreads();
      vbase += dc_region_doubles(K, t);
    }
    if (run && tid < K) dg[tid] *= scale;
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
    newcol[i] = (unsigned char)pos;
    gst(&a.lam[pos], fmax(li, 0.0));
    if (!isfinite(li)) atomicOr(&st->flags, 2u);
  }
  if (tid == 0) {   // the secular-equation counters of the merges
    atomicMax(&st->pad, min(sh_maxit, 255));
    if (sh_noconv) atomicOr(&st->flags, 8u);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int r = rl + 16 * i, c = cg + 16 * q;
      if (r < K && c < K) gst(&a.Q[r * K + newcol[c]], Z[i][q]);
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
