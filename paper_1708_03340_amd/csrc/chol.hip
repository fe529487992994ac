// Cholesky steps of CholeskyQR2, one workgroup of 256 threads per tree node,
// the node's K x K Gram matrix in LDS (K <= 128, padded to whole 16 x 16
// blocks with an identity).
//
// Section 3.4 asks for a reduced QR of every leaf frame and of M_{2,3}(B_t);
// CholeskyQR2 gets R from two Gram matrices: G = W^T W = R1^T R1, then
// G2 = (W R1^{-1})^T (W R1^{-1}) = R2^T R2 and R = R2 R1.
//  * sweep 1 factors G + s I, s a small multiple of the rounding error of G
//    (shifted CholeskyQR, Fukaya et al. 2020), and clamps pivots that still
//    fall below tol; the second sweep repairs R;
//  * sweep 2 drops the rows whose pivot vanishes (rank-deficient frames such
//    as those of the sum A + A) and flags them.
//
// Right-looking blocked factorisation, blocks of 16.  For each block column
// p: wave 0 factors the diagonal block in registers (left-looking, one
// pivot at a time) and inverts its factor; the block row R_pq = R_pp^{-T} A_pq and the symmetric
// trailing update A_qr -= R_pq^T R_pr are float64 MFMA 16x16x4 products
// spread over the four waves.  R^{-1} is then formed by blocked back
// substitution, X_pq = -X_pp sum_{k=p+1..q} R_pk X_kq, also on MFMA.  A
// dropped row is a zero row of R and a unit row of the matrix inverted.
//
// Sweep 2 ends with the step's combination, R = R2 R1 and
// R^{-1} = R1^{-1} R2^{-1} (products of block upper-triangular matrices on
// MFMA, R2 and R2^{-1} from LDS, R1 and R1^{-1} from global memory), and
// normalises R by 2^-e, e the binary exponent of max |R|; e is added to the
// tensor's scale exponent and Rf receives R in the forward-product type.
#include "dense_util.h"

namespace ht {
namespace {

constexpr int NT = DNT;
constexpr int LDL = KMAX + 1;   // LDS row stride of the matrix
constexpr int LDD = 17;         // LDS row stride of a 16 x 16 block inverse

typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ doublex4 mfma(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// sweep 1: G -> R1, Ri1 = R1^{-1}.  sweep 2: G2 -> R2 (rows of vanishing
// pivots dropped) and R2^{-1} (unit diagonal on dropped rows), kept in LDS,
// then R, Ri and Rf as above.
__global__ __launch_bounds__(NT) void chol_kernel(const SmallArgs* __restrict__ args, int sweep,
                                                  GlobalState* st) {
  __shared__ double L[KMAX * LDL];            // A, then R (upper blocks) and X^T (lower blocks)
  __shared__ double Xd[KMAX / 16][16 * LDD];  // inverses of the diagonal blocks of R
  __shared__ double red[NT / 64];
  __shared__ int dropped[KMAX];
  __shared__ int any;
  const SmallArgs& a = args[blockIdx.x];
  if (a.st) st = a.st;
  const int K = a.K;
  const int NB = (K + 15) >> 4, Kp = NB * 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wv = __builtin_amdgcn_readfirstlane(wave);   // the same, in a scalar register
  const int l16 = lane & 15, l4 = lane >> 4;
  const double* Gin = sweep == 1 ? a.G : a.G2;
  bool bad = false;
  // wave w loads rows w, w + 4, ...; lane c columns c and c + 64; sixteen
  // rows in flight per wave
  for (int r0 = wave; r0 < Kp; r0 += 64) {
    double v[16][2];
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // every load is issued (clamped address, masked value): a guarded
        // load would wait for each one in turn; identity on the padding
        const int r = r0 + 4 * u, c = lane + 64 * h;
        const bool in = r < K && c < K;
        const double g = gld(&Gin[min(r, K - 1) * K + min(c, K - 1)]);
        v[u][h] = g * (in ? 1.0 : 0.0) + ((!in && r == c) ? 1.0 : 0.0);
      }
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = r0 + 4 * u, c = lane + 64 * h;
        if (r < Kp && c < Kp) {
          if (!isfinite(v[u][h])) bad = true;
          L[r * LDL + c] = v[u][h];
        }
      }
  }
  for (int i = tid; i < KMAX; i += NT) dropped[i] = 0;
  if (tid == 0) any = 0;
  __syncthreads();
  double md = 0.0, tr = 0.0;
  for (int i = tid; i < K; i += NT) {
    const double v = L[i * LDL + i];
    if (isfinite(v)) {
      md = fmax(md, v);
      tr += fmax(v, 0.0);
    }
  }
  double maxd = wg_max(md, red);
  const double badany = wg_max(bad ? 1.0 : 0.0, red);
  if (badany > 0.0 && tid == 0) atomicOr(&st->flags, 2u);
  if (sweep == 1 && a.shift_rel > 0.0) {
    // shifted first sweep: R1^T R1 = G + s I with s above the rounding error
    // of G and of the factorisation, so that ||W R1^{-1}|| stays near 1 when
    // W is rank-deficient or ill-conditioned (an unshifted factor of such a
    // G can have an inverse of any size); the second sweep restores R
    const double s = a.shift_rel * wg_sum(tr, red);
    for (int i = tid; i < K; i += NT) L[i * LDL + i] += s;
    maxd += s;
    __syncthreads();
  }
  const double tol = maxd > 0.0 ? a.tol_rel * maxd : 1.0;

  for (int p = 0; p < NB; ++p) {
    double* D = &L[16 * p * LDL + 16 * p];
    // ---- diagonal block, by wave 0 in registers, left-looking: lane r
    // (mod 16) owns column r of the block, A_jr for j <= r taken from the
    // upper triangle (the only one the trailing updates keep), and builds
    // column r of R_pp.  Step j forms lane r's entry of column j of the
    // Schur complement, s_r = A_jr - sum_{i<j} R_ir R_ij (R_ij from lane j
    // by a DPP row broadcast), takes the pivot s_j from lane j and sets
    // R_jr = s_r / sqrt(s_j).  Every entry is formed once, so no symmetric
    // copy can drift, and the pivot chain waits only on the last term of
    // each sum.  X_pp = R_pp^{-1} follows by column-oriented back
    // substitution.
    if (wave == 0) {
      const int r = l16;
      double rc[16];      // rc[j] = R_jr (0 below the diagonal)
      double s[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) s[j] = j <= r ? D[j * LDL + r] : 0.0;
      double rinv = 1.0;  // 1 / R_rr; 1 on a dropped row (a unit row of the inverse)
      unsigned dmask = 0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double sj = s[j];
#pragma unroll
        for (int i = 0; i < j; ++i) sj = fma(-rc[i], row16_bcast(rc[i], j), sj);
        const double pj = row16_bcast(sj, j);
        // branch-free pivot rule: padding takes 1; a pivot not above tol is
        // clamped to tol in sweep 1 and dropped in sweep 2 (a zero row of R
        // that updates nothing)
        const bool pad = 16 * p + j >= K;
        const bool small = !(pj > tol);
        const bool drop = !pad && small && sweep != 1;
        const double pv = pad ? 1.0 : (small ? (sweep == 1 ? tol : 1.0) : pj);
        dmask |= drop ? (1u << j) : 0u;
        const double rj = rsqrt_nr(pv);
        const double v = r > j ? sj * rj : (r == j ? pv * rj : 0.0);
        rc[j] = drop ? 0.0 : v;
        if (r == j) rinv = drop ? 1.0 : rj;
      }
      if (lane < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) D[i * LDL + r] = rc[i];
        dropped[16 * p + r] = (dmask >> r) & 1u;
        if (lane == 0 && dmask) any = 1;
      }
      // X_pp: lane c forms column c, x = e_c, then for k = 15 .. 0:
      // x_k /= R_kk, x_i -= R_ik x_k (i < k), R_ik from lane k
      {
        const int c = l16;
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] = i == c ? 1.0 : 0.0;
#pragma unroll
        for (int k = 15; k >= 0; --k) {
          x[k] *= row16_bcast(rinv, k);
#pragma unroll
          for (int i = 0; i < k; ++i) x[i] = fma(-row16_bcast(rc[i], k), x[k], x[i]);
        }
        if (lane < 16) {
#pragma unroll
          for (int i = 0; i < 16; ++i) Xd[p][i * LDD + c] = x[i];
        }
      }
    }
    __syncthreads();
    // ---- block row: R_pq = X_pp^T A_pq, dropped rows zeroed
    for (int q = p + 1 + wave; q < NB; q += 4) {
      doublex4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + l4;
        acc = mfma(Xd[p][k * LDD + l16], L[(16 * p + k) * LDL + 16 * q + l16], acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + l4;
        L[(16 * p + r) * LDL + 16 * q + l16] = dropped[16 * p + r] ? 0.0 : acc[v];
      }
    }
    __syncthreads();
    // ---- trailing update of the upper blocks: A_qr -= R_pq^T R_pr, p < q <= r
    {
      const int nt = NB - 1 - p;
      int idx = 0;
      for (int q = p + 1; q < NB; ++q)
        for (int r = q; r < NB; ++r, ++idx) {
          if ((idx & 3) != wave) continue;
          doublex4 acc;
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[v] = L[(16 * q + 4 * v + l4) * LDL + 16 * r + l16];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = 16 * p + 4 * s + l4;
            acc = mfma(-L[k * LDL + 16 * q + l16], L[k * LDL + 16 * r + l16], acc);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) L[(16 * q + 4 * v + l4) * LDL + 16 * r + l16] = acc[v];
        }
      (void)nt;
    }
    __syncthreads();
  }

  // ---- R1 out (upper blocks of L; zero below the diagonal)
  if (sweep == 1)
    for (int r = wave; r < K; r += NT / 64)
      for (int c = lane; c < K; c += 64) {
        const double lv = L[r * LDL + c];
        gst(&a.R1[r * K + c], lv * (c >= r ? 1.0 : 0.0));
      }
  __syncthreads();   // the lower blocks of L are overwritten below

  // ---- X = R^{-1} by blocked back substitution; X_pq (p < q) is kept
  // transposed in the lower block (q, p) of L, X_pp in Xd[p]
  for (int p = NB - 2; p >= 0; --p) {
    for (int q = p + 1 + wave; q < NB; q += 4) {
      // S = sum_{k=p+1..q} R_pk X_kq
      doublex4 sacc = {0, 0, 0, 0};
      for (int k = p + 1; k <= q; ++k) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int kk = 4 * s + l4;
          const double ra = L[(16 * p + l16) * LDL + 16 * k + kk];
          const double xb = k == q ? Xd[q][kk * LDD + l16] : L[(16 * q + l16) * LDL + 16 * k + kk];
          sacc = mfma(ra, xb, sacc);
        }
      }
      // X_pq = -X_pp S: the accumulator layout of S is the B operand layout
      doublex4 xacc = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) xacc = mfma(-Xd[p][l16 * LDD + 4 * s + l4], sacc[s], xacc);
#pragma unroll
      for (int v = 0; v < 4; ++v) L[(16 * q + l16) * LDL + 16 * p + 4 * v + l4] = xacc[v];
    }
    __syncthreads();
  }
  if (sweep == 1) {
    for (int r = wave; r < K; r += NT / 64)
      for (int c = lane; c < K; c += 64) {
        const int pr = r >> 4, pc = c >> 4;
        const double xd = Xd[pr][(r & 15) * LDD + (c & 15)], lv = L[c * LDL + r];
        gst(&a.Ri1[r * K + c], xd * (pr == pc ? 1.0 : 0.0) + lv * (pr < pc ? 1.0 : 0.0));
      }
    return;
  }
  if (any && tid == 0) atomicOr(&st->flags, 1u);

  // ---- sweep 2: R = R2 R1 and Ri = R1^{-1} R2^{-1} (products of block
  // upper-triangular matrices).  Wave w takes the block columns w and
  // NBMAX - 1 - w of R, R_pq = sum_{k=p..q} R2_pk R1_kq: it loads each column
  // of R1 once (all loads of a column in flight together) and keeps the
  // column's blocks in registers until the power-of-two normalisation is
  // known.  Then it takes the block rows w and NBMAX - 1 - w of Ri,
  // Ri_pq = sum_{k=p..q} Ri1_pk X_kq, from one load of the row of Ri1.  In
  // both products the blocks of a row or column are advanced together for
  // each k, so consecutive MFMAs feed different accumulators.
  constexpr int NBMAX = KMAX / 16;
  // the node's pointers in locals (the stores would otherwise make the
  // compiler reload them from the argument table)
  const double* const R1g = a.R1;
  const double* const Ri1g = a.Ri1;
  double* const Rg = a.R;
  double* const Rig = a.Ri;
  void* const Rfg = a.Rf;
  const bool rf32 = a.rf_type == F32;
  double mx = 0.0;
  doublex4 acc[2][NBMAX];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = u == 0 ? wv : NBMAX - 1 - wv;
#pragma unroll
    for (int p = 0; p < NBMAX; ++p) acc[u][p] = doublex4{0.0, 0.0, 0.0, 0.0};
    if (q >= NB) continue;
    double b1[NBMAX][4];   // R1_kq, B operand layout
#pragma unroll
    for (int k = 0; k < NBMAX; ++k)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kr = 16 * k + 4 * s + l4, c = 16 * q + l16;
        const double x = gld(&R1g[min(kr, K - 1) * K + min(c, K - 1)]);
        b1[k][s] = (k <= q && kr < K && c < K) ? x : 0.0;
      }
#pragma unroll
    for (int k = 0; k < NBMAX; ++k) {
      if (k > q) break;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = 4 * s + l4;
#pragma unroll
        for (int p = 0; p <= k; ++p) {
          const double r2 = L[(16 * p + l16) * LDL + 16 * k + kk] * ((k > p || kk >= l16) ? 1.0 : 0.0);
          acc[u][p] = mfma(r2, b1[k][s], acc[u][p]);
        }
      }
    }
#pragma unroll
    for (int p = 0; p < NBMAX; ++p)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * p + 4 * v + l4, c = 16 * q + l16;
        if (p <= q && r < K && c < K) mx = fmax(mx, fabs(acc[u][p][v]));
      }
  }
  const int e = exp2_of(wg_max(mx, red));
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = u == 0 ? wv : NBMAX - 1 - wv;
    if (q >= NB) continue;
#pragma unroll
    for (int p = 0; p < NBMAX; ++p) {
      if (p > q) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * p + 4 * v + l4, c = 16 * q + l16;
        if (r < K && c < K) {
          const double y = ldexp(acc[u][p][v], -e);
          gst(&Rg[r * K + c], y);
          if (rf32) reinterpret_cast<float*>(Rfg)[r * K + c] = (float)y;
          else reinterpret_cast<double*>(Rfg)[r * K + c] = y;
        }
      }
    }
  }
  // blocks below the diagonal are zero
  for (int r = wave; r < K; r += NT / 64)
    for (int c = lane; c < (r & ~15); c += 64) {
      gst(&Rg[r * K + c], 0.0);
      gst(&Rig[r * K + c], 0.0);
      if (rf32) reinterpret_cast<float*>(Rfg)[r * K + c] = 0.0f;
      else reinterpret_cast<double*>(Rfg)[r * K + c] = 0.0;
    }
#pragma unroll 1
  for (int u = 0; u < 2; ++u) {
    const int p = u == 0 ? wv : NBMAX - 1 - wv;
    if (p >= NB) continue;
    double a1[NBMAX][4];   // Ri1_pk, A operand layout
#pragma unroll
    for (int k = 0; k < NBMAX; ++k)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int r = 16 * p + l16, kc = 16 * k + 4 * s + l4;
        const double x = gld(&Ri1g[min(r, K - 1) * K + min(kc, K - 1)]);
        a1[k][s] = (k >= p && r < K && kc < K) ? x : 0.0;
      }
    doublex4 iacc[NBMAX];
#pragma unroll
    for (int q = 0; q < NBMAX; ++q) iacc[q] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NBMAX; ++k) {
      if (k >= NB) break;
      if (k < p) continue;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = 4 * s + l4;
#pragma unroll
        for (int q = k; q < NBMAX; ++q) {
          const double xb = k == q ? Xd[q][kk * LDD + l16] : L[(16 * q + l16) * LDL + 16 * k + kk];
          iacc[q] = mfma(a1[k][s], xb, iacc[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NBMAX; ++q) {
      if (q >= NB) break;
      if (q < p) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * p + 4 * v + l4, c = 16 * q + l16;
        if (r < K && c < K) gst(&Rig[r * K + c], iacc[q][v]);
      }
    }
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


}  // namespace ht
