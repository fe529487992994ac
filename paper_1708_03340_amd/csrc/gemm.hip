// Strided, batched, segmented GEMM on the gfx950 matrix cores.
//
// Every contraction of the truncation is one of these: frame Grams U^T U,
// mode-1/2/3 products (X,Y,Z) o B on row-major transfer tensors, the Gramian
// contractions of eqs. (acctransferSon1/2) and the projections of
// eq. (transfertransformationtrunc).  A 64x64 output tile per workgroup of four
// wave64s (each wave owns 32x32 = 2x2 MFMA 16x16 blocks); the reduction is
// staged through LDS in k-slabs of 16 with a register prefetch of the next
// slab.  Operands are converted to the MFMA type when they are written to LDS,
// so float32 data feeds the FP64 matrix cores exactly.
#include "ht_internal.h"

namespace ht {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

template <typename T> struct AccOf;
template <> struct AccOf<float> { using V = floatx4; };
template <> struct AccOf<double> { using V = doublex4; };

__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Reduction cursor over segments / reduction blocks.
struct Cursor {
  int seg;   // current segment
  int k0;    // offset inside the segment
};

template <typename TA, typename TB, typename TM, bool ACC64>
__global__ __launch_bounds__(NT) void gemm_kernel(const GemmDesc* __restrict__ descs, int maxbatch,
                                                  int splitk, int tC, int mode, int aK, int bK) {
  __shared__ TM As[BK][BM + 4];
  __shared__ TM Bs[BK][BN + 4];

  const GemmDesc& D = descs[blockIdx.z / maxbatch];
  const int b = blockIdx.z % maxbatch;
  if (b >= D.nbatch) return;
  const int M = D.M, N = D.N;
  const int tilesN = (N + BN - 1) / BN;
  const int tilesM = (M + BM - 1) / BM;
  if ((int)blockIdx.x >= tilesM * tilesN) return;
  const int tm = blockIdx.x / tilesN, tn = blockIdx.x % tilesN;

  const int nseg = D.nseg > 0 ? D.nseg : D.KB;
  auto segK = [&](int s) -> int { return D.nseg > 0 ? D.segK[s] : D.K; };
  int total = 0;
  for (int s = 0; s < nseg; ++s) total += (segK(s) + BK - 1) / BK;
  const int per = (total + splitk - 1) / splitk;
  const int t0 = blockIdx.y * per;
  const int t1 = min(total, t0 + per);
  if (t0 >= t1 && !(mode == GEMM_STORE && blockIdx.y == 0)) return;

  const TA* Ab = reinterpret_cast<const TA*>(D.A);
  const TB* Bb = reinterpret_cast<const TB*>(D.B);
  const int64_t aoff_b = (int64_t)b * D.sAb, boff_b = (int64_t)b * D.sBb;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // thread -> (row, k) coordinates of its four loaded elements
  int a_r[4], a_k[4], b_c[4], b_k[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (aK) { a_r[i] = tid >> 2; a_k[i] = (tid & 3) * 4 + i; }
    else    { a_r[i] = (tid & 15) * 4 + i; a_k[i] = tid >> 4; }
    if (bK) { b_c[i] = tid >> 2; b_k[i] = (tid & 3) * 4 + i; }
    else    { b_c[i] = (tid & 15) * 4 + i; b_k[i] = tid >> 4; }
  }

  // locate tile t0
  Cursor cur{0, 0};
  {
    int skip = t0;
    while (cur.seg < nseg) {
      int nt = (segK(cur.seg) + BK - 1) / BK;
      if (skip < nt) { cur.k0 = skip * BK; break; }
      skip -= nt;
      cur.seg++;
    }
  }

  TM ra[4], rb[4];
  auto load = [&](const Cursor& c) {
    const int s = c.seg;
    const int ks = segK(s);
    const TA* Ap = (D.nseg > 0 ? reinterpret_cast<const TA*>(D.segA[s]) : Ab + (int64_t)s * D.sAkb) + aoff_b;
    const TB* Bp = Bb + (D.nseg > 0 ? D.segBoff[s] : (int64_t)s * D.sBkb) + boff_b;
    const int64_t sAk = D.nseg > 0 ? D.segAk[s] : D.sAk;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // loads go to a clamped in-range address and the value is multiplied
      // by a 0/1 mask: a guarded load (or a select on its value) is compiled
      // into a branch that waits for the load before the next one is issued.
      // A clamped element only meets the mask outside the valid range of the
      // output or on a k index whose true term is in the sum anyway, so a
      // non-finite input still reaches every valid output it belongs to.
      const int gm = tm * BM + a_r[i], gk = c.k0 + a_k[i];
      const int cm = min(gm, M - 1), ck = min(gk, ks - 1);
      TM va;
      if (D.kr) va = (TM)(gld(&D.krY1[(int64_t)cm * D.krld1 + ck / D.krK2]) * gld(&D.krY2[(int64_t)cm * D.krld2 + ck % D.krK2]));
      else va = (TM)gld(&Ap[(int64_t)cm * D.sAm + (int64_t)ck * sAk]);
      ra[i] = va * (TM)(gm < M && gk < ks);
      const int gn = tn * BN + b_c[i], gkb = c.k0 + b_k[i];
      const TM vb = (TM)gld(&Bp[(int64_t)min(gkb, ks - 1) * D.sBk + (int64_t)min(gn, N - 1) * D.sBn]);
      rb[i] = vb * (TM)(gn < N && gkb < ks);
    }
  };
  auto advance = [&](Cursor& c) {
    c.k0 += BK;
    if (c.k0 >= segK(c.seg)) { c.seg++; c.k0 = 0; }
    while (c.seg < nseg && segK(c.seg) == 0) c.seg++;
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      As[a_k[i]][a_r[i]] = ra[i];
      Bs[b_k[i]][b_c[i]] = rb[i];
    }
  };

  using V = typename AccOf<TM>::V;
  V acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = V{0, 0, 0, 0};
  // ACC64: the float32 MFMA accumulator is emptied into float64 registers
  // after every k-slab, so rounding grows with the slab (16), not with K
  doublex4 acc64[2][2];
  if (ACC64) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc64[i][j] = doublex4{0, 0, 0, 0};
  }

  if (t0 < t1) {
    load(cur);
    stash();
    __syncthreads();
    for (int it = t0; it < t1; ++it) {
      const bool more = it + 1 < t1;
      if (more) { advance(cur); load(cur); }
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
        const TM a0 = As[kr][wm * 32 + (lane & 15)];
        const TM a1 = As[kr][wm * 32 + 16 + (lane & 15)];
        const TM b0 = Bs[kr][wn * 32 + (lane & 15)];
        const TM b1 = Bs[kr][wn * 32 + 16 + (lane & 15)];
        acc[0][0] = mfma16(a0, b0, acc[0][0]);
        acc[0][1] = mfma16(a0, b1, acc[0][1]);
        acc[1][0] = mfma16(a1, b0, acc[1][0]);
        acc[1][1] = mfma16(a1, b1, acc[1][1]);
      }
      if (ACC64) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              acc64[i][j][v] += (double)acc[i][j][v];
              acc[i][j][v] = (TM)0;
            }
      }
      __syncthreads();
      if (more) {
        stash();
        __syncthreads();
      }
    }
  }

  double alpha = D.alpha;
  if (D.alpha_dev) alpha *= gld(D.alpha_dev);
  char* Cb = reinterpret_cast<char*>(D.C);
  const int esz = tC == F64 ? 8 : 4;
  const int64_t coff_b = (int64_t)b * D.sCb;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // accumulator register v of lane l: FP32 16x16x4 holds rows 4(l/16)+v,
        // FP64 16x16x4 holds rows 4v + l/16 (both in column l%16)
        const int rin = sizeof(TM) == 8 ? v * 4 + (lane >> 4) : (lane >> 4) * 4 + v;
        const int row = tm * BM + wm * 32 + i * 16 + rin;
        const int col = tn * BN + wn * 32 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          const double val = alpha * (ACC64 ? acc64[i][j][v] : (double)acc[i][j][v]);
          const int64_t off = coff_b + (int64_t)row * D.sCm + (int64_t)col * D.sCn;
          if (tC == F64) {
            double* p = reinterpret_cast<double*>(Cb) + off;
            if (mode == GEMM_ATOMIC) gatomic_add(p, val); else gst(p, val);
          } else {
            float* p = reinterpret_cast<float*>(Cb) + off;
            if (mode == GEMM_ATOMIC) gatomic_add(p, (float)val); else gst(p, (float)val);
          }
        }
      }
  (void)esz;
}

template <typename TA, typename TB, typename TM, bool ACC64 = false>
hipError_t go(const GemmLaunch& g, hipStream_t s) {
  dim3 grid(g.maxtiles, g.splitk, g.ndesc * g.maxbatch);
  hipLaunchKernelGGL((gemm_kernel<TA, TB, TM, ACC64>), grid, dim3(NT), 0, s, g.descs, g.maxbatch, g.splitk,
                     g.tC, g.mode, g.a_kcontig ? 1 : 0, g.b_kcontig ? 1 : 0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ 128 x 128 float64 tiles
// For the large float64 contractions: 128 x 128 output tile per workgroup,
// four waves of 64 x 64 (4 x 4 MFMA 16x16x4 blocks: 16 MFMAs per 8 LDS
// fragment reads), k-slabs of 16 double-buffered in LDS (one barrier per
// slab) with the next slab prefetched into registers while the current one
// is multiplied.  Operands of any type are widened to float64 on the way
// into LDS.
constexpr int BT = 128, PADT = 4;

template <typename TA, typename TB>
__global__ __launch_bounds__(NT, 2) void gemm128_kernel(const GemmDesc* __restrict__ descs, int maxbatch,
                                                       int splitk, int tC, int mode, int aK, int bK) {
  __shared__ double As[2][BK][BT + PADT];
  __shared__ double Bs[2][BK][BT + PADT];

  const GemmDesc& D = descs[blockIdx.z / maxbatch];
  const int b = blockIdx.z % maxbatch;
  if (b >= D.nbatch) return;
  const int M = D.M, N = D.N;
  const int tilesN = (N + BT - 1) / BT;
  const int tilesM = (M + BT - 1) / BT;
  if ((int)blockIdx.x >= tilesM * tilesN) return;
  const int tm = blockIdx.x / tilesN, tn = blockIdx.x % tilesN;

  const int nseg = D.nseg > 0 ? D.nseg : D.KB;
  auto segK = [&](int s) -> int { return D.nseg > 0 ? D.segK[s] : D.K; };
  int total = 0;
  for (int s = 0; s < nseg; ++s) total += (segK(s) + BK - 1) / BK;
  const int per = (total + splitk - 1) / splitk;
  const int t0 = blockIdx.y * per;
  const int t1 = min(total, t0 + per);
  if (t0 >= t1 && !(mode == GEMM_STORE && blockIdx.y == 0)) return;

  const TA* Ab = reinterpret_cast<const TA*>(D.A);
  const TB* Bb = reinterpret_cast<const TB*>(D.B);
  const int64_t aoff_b = (int64_t)b * D.sAb, boff_b = (int64_t)b * D.sBb;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // each thread moves 8 elements of A and 8 of B per slab
  //   k-contiguous operand: row r = tid/2, k = (tid%2)*8 + i
  //   row-contiguous operand: k = tid/16, row r = (tid%16)*8 + i
  const int a_r0 = aK ? (tid >> 1) : (tid & 15) * 8;
  const int a_k0 = aK ? (tid & 1) * 8 : (tid >> 4);
  const int b_r0 = bK ? (tid >> 1) : (tid & 15) * 8;
  const int b_k0 = bK ? (tid & 1) * 8 : (tid >> 4);

  Cursor cur{0, 0};
  {
    int skip = t0;
    while (cur.seg < nseg) {
      int nt = (segK(cur.seg) + BK - 1) / BK;
      if (skip < nt) { cur.k0 = skip * BK; break; }
      skip -= nt;
      cur.seg++;
    }
  }

  double ra[8], rb[8];
  auto load = [&](const Cursor& c) {
    const int s = c.seg;
    const int ks = segK(s);
    const TA* Ap = (D.nseg > 0 ? reinterpret_cast<const TA*>(D.segA[s]) : Ab + (int64_t)s * D.sAkb) + aoff_b;
    const TB* Bp = Bb + (D.nseg > 0 ? D.segBoff[s] : (int64_t)s * D.sBkb) + boff_b;
    const int64_t sAk = D.nseg > 0 ? D.segAk[s] : D.sAk;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = aK ? a_r0 : a_r0 + i, k = aK ? a_k0 + i : a_k0;
      const int gm = tm * BT + r, gk = c.k0 + k;
      const double va = (double)gld(&Ap[(int64_t)min(gm, M - 1) * D.sAm + (int64_t)min(gk, ks - 1) * sAk]);
      ra[i] = va * (double)(gm < M && gk < ks);   // clamped load, 0/1 mask
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = bK ? b_r0 : b_r0 + i, k = bK ? b_k0 + i : b_k0;
      const int gn = tn * BT + r, gk = c.k0 + k;
      const double vb = (double)gld(&Bp[(int64_t)min(gk, ks - 1) * D.sBk + (int64_t)min(gn, N - 1) * D.sBn]);
      rb[i] = vb * (double)(gn < N && gk < ks);
    }
  };
  auto advance = [&](Cursor& c) {
    c.k0 += BK;
    if (c.k0 >= segK(c.seg)) { c.seg++; c.k0 = 0; }
    while (c.seg < nseg && segK(c.seg) == 0) c.seg++;
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (aK) As[buf][a_k0 + i][a_r0] = ra[i]; else As[buf][a_k0][a_r0 + i] = ra[i];
      if (bK) Bs[buf][b_k0 + i][b_r0] = rb[i]; else Bs[buf][b_k0][b_r0 + i] = rb[i];
    }
  };

  doublex4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0, 0, 0, 0};

  if (t0 < t1) {
    load(cur);
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int it = t0; it < t1; ++it) {
      const bool more = it + 1 < t1;
      if (more) { advance(cur); load(cur); }
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
        double fa[4], fb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          fa[i] = As[buf][kr][wm * 64 + i * 16 + (lane & 15)];
          fb[i] = Bs[buf][kr][wn * 64 + i * 16 + (lane & 15)];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = mfma16(fa[i], fb[j], acc[i][j]);
      }
      if (more) {
        stash(buf ^ 1);
        buf ^= 1;
      }
      __syncthreads();
    }
  }

  double alpha = D.alpha;
  if (D.alpha_dev) alpha *= gld(D.alpha_dev);
  char* Cb = reinterpret_cast<char*>(D.C);
  const int64_t coff_b = (int64_t)b * D.sCb;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // FP64 16x16x4: register v of lane l holds row 4v + l/16, column l%16
        const int row = tm * BT + wm * 64 + i * 16 + v * 4 + (lane >> 4);
        const int col = tn * BT + wn * 64 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          const double val = alpha * acc[i][j][v];
          const int64_t off = coff_b + (int64_t)row * D.sCm + (int64_t)col * D.sCn;
          if (tC == F64) {
            double* p = reinterpret_cast<double*>(Cb) + off;
            if (mode == GEMM_ATOMIC) gatomic_add(p, val); else gst(p, val);
          } else {
            float* p = reinterpret_cast<float*>(Cb) + off;
            if (mode == GEMM_ATOMIC) gatomic_add(p, (float)val); else gst(p, (float)val);
          }
        }
      }
}

template <typename TA, typename TB>
hipError_t go128(const GemmLaunch& g, hipStream_t s) {
  dim3 grid(g.maxtiles, g.splitk, g.ndesc * g.maxbatch);
  hipLaunchKernelGGL((gemm128_kernel<TA, TB>), grid, dim3(NT), 0, s, g.descs, g.maxbatch, g.splitk, g.tC,
                     g.mode, g.a_kcontig ? 1 : 0, g.b_kcontig ? 1 : 0);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm(const GemmLaunch& g, hipStream_t s) {
  if (g.ndesc <= 0 || g.maxtiles <= 0) return hipSuccess;
  if (g.sb) return launch_gemm_sb(g, s);
  if (g.rk) return launch_gemm_rk(g, s);
  const bool a32 = g.tA == F32, b32 = g.tB == F32;
  if (g.big) {
    if (a32 && b32) return go128<float, float>(g, s);
    if (a32 && !b32) return go128<float, double>(g, s);
    if (!a32 && b32) return go128<double, float>(g, s);
    return go128<double, double>(g, s);
  }
  if (g.math == MATH_F32 && g.acc64) {
    if (a32 && b32) return go<float, float, float, true>(g, s);
    if (a32 && !b32) return go<float, double, float, true>(g, s);
    if (!a32 && b32) return go<double, float, float, true>(g, s);
    return go<double, double, float, true>(g, s);
  }
  if (g.math == MATH_F32) {
    if (a32 && b32) return go<float, float, float>(g, s);
    if (a32 && !b32) return go<float, double, float>(g, s);
    if (!a32 && b32) return go<double, float, float>(g, s);
    return go<double, double, float>(g, s);
  }
  if (a32 && b32) return go<float, float, double>(g, s);
  if (a32 && !b32) return go<float, double, double>(g, s);
  if (!a32 && b32) return go<double, float, double>(g, s);
  return go<double, double, double>(g, s);
}

}  // namespace ht
