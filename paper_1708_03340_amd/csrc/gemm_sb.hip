// Float64 products of a small matrix with a long streamed one,
//   C[m][n] = alpha * sum_k S[m][k] * T[k][n],   m < Ms <= 128, k < Kt <= 128,
// the shape of most contractions of the truncation: the CholeskyQR2 factor
// products Y = R^{-T} M1(B') and Qo = R^{-T} M1(B') (Section 3.4), the first
// Gramian contraction C = Bhat_t M1(Qo) (eqs. (acctransferSon1/2)), the mode-1
// and mode-2 projections (eq. (transfertransformationtrunc)) and, transposed,
// the leaf frame products W R^{-1} and W (R^{-1} Q|).
//
// A workgroup keeps S whole in LDS (zero-padded to 128 x 128) and walks a
// strip of 128-column tiles of T.  Each wave owns 32 columns of a tile and all
// rows: 8 x 2 MFMA 16x16x4 blocks per 4-deep k step.  T never passes through
// LDS: each lane loads its MFMA operand straight from HBM, one 32-deep chunk
// ahead of the chunk being multiplied, so the loads of a tile overlap the
// products of the previous chunk.  S is reloaded only when the batch changes
// and S has a batch stride.
//
// Reductions of 97 .. 128 use gemm_sb_ring_kernel below (four operand
// buffers, loads two chunks ahead).
//
// GemmDesc mapping (swap = 0): S = A (M x K), T = B (K x N), C as given.
// swap = 1: S = B^T (N x K), T = A^T (K x M), out[m][n] = C[n][m]: the small
// operand is B and A is streamed along M.  Segments (GemmDesc::nseg) split
// the reduction; each has its own A pointer and k stride and a B offset.
#include "ht_internal.h"

namespace ht {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int SB_K = 128;          // largest reduction length
constexpr int SB_MP = 128 + 4;     // LDS row length of S (padded)
constexpr int SB_TN = 128;         // streamed columns per tile

// Sink for the stores of lanes outside the result (never read): with it every
// lane stores, and no store sits behind a branch.
__device__ double g_sb_sink[512];

template <typename T>
__device__ __forceinline__ double ld_as_double(const char* p) {
  return (double)gld(reinterpret_cast<const T*>(p));
}

// NRB: row blocks of 16 that hold rows of S (2, 4, 6 or 8); the MFMAs of
// the blocks past them are not issued.
template <typename TS, typename TT, int WN, int CD, int NRB>
__global__ __launch_bounds__(512 / WN, 1) void gemm_sb_kernel(const GemmDesc* __restrict__ descs, int swap,
                                                             int tC) {
  constexpr int SB_NT = 512 / WN;     // 8 / WN waves, each 16 * WN columns of a 128-column tile
  constexpr int KS = CD / 4;          // 4-deep MFMA steps per chunk (CD = chunk depth, 32 or 64)
  __shared__ double Ss[SB_K][SB_MP];
  __shared__ const char* trow[SB_K];   // byte address of T[k][0] (batch 0)
  __shared__ const char* srow[SB_K];   // byte address of S[0][k] (batch 0)

  const GemmDesc& D = descs[blockIdx.y];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int Ms = swap ? D.N : D.M;
  const int Ns = swap ? D.M : D.N;
  const int nseg = D.nseg > 0 ? D.nseg : 1;
  const int esS = sizeof(TS), esT = sizeof(TT);
  // strides in bytes
  const int64_t s_m = (swap ? D.sBn : D.sAm) * esS;          // S row (m) stride
  const int64_t t_n = (swap ? D.sAm : D.sBn) * esT;          // T column (n) stride
  const int64_t s_b = (swap ? D.sBb : D.sAb) * esS;          // batch strides
  const int64_t t_b = (swap ? D.sAb : D.sBb) * esT;
  const int64_t c_m = swap ? D.sCn : D.sCm, c_n = swap ? D.sCm : D.sCn;

  // per-k row tables; k past the reduction points at the last row (S is zero there)
  int Kt = 0;
  for (int s = 0; s < nseg; ++s) Kt += D.nseg > 0 ? D.segK[s] : D.K;
  if (tid < SB_K) {
    const int k = min(tid, Kt - 1);
    int s = 0, kofs = 0;
    while (s + 1 < nseg && k >= kofs + (D.nseg > 0 ? D.segK[s] : D.K)) {
      kofs += D.nseg > 0 ? D.segK[s] : D.K;
      ++s;
    }
    const int kl = k - kofs;
    const char* Aseg = reinterpret_cast<const char*>(D.nseg > 0 ? D.segA[s] : D.A);
    const int64_t sAk = D.nseg > 0 ? D.segAk[s] : D.sAk;
    const int64_t boff = D.nseg > 0 ? D.segBoff[s] : 0;
    const char* Bb = reinterpret_cast<const char*>(D.B);
    if (!swap) {
      srow[tid] = Aseg + kl * sAk * esS;
      trow[tid] = Bb + (boff + kl * D.sBk) * esT;
    } else {
      srow[tid] = Bb + (boff + kl * D.sBk) * esS;
      trow[tid] = Aseg + kl * sAk * esT;
    }
  }
  const int Kp = (Kt + CD - 1) / CD * CD;  // reduction padded to whole chunks
  const int nchunk = Kp / CD;
  const int tilesN = (Ns + SB_TN - 1) / SB_TN;
  const int nitems = tilesN * D.nbatch;
  double alpha = D.alpha;
  if (D.alpha_dev) alpha *= gld(D.alpha_dev);

  // S into LDS: thread tid owns column tid % 128 and every (SB_NT / 128)-th
  // row; all its loads are issued before the first store (clamped addresses,
  // masked values: rows past Kt point at row Kt - 1), so the fill waits on
  // one memory latency, not one per element
  auto load_S = [&](int b) {
    __syncthreads();   // previous users of Ss are done; the row tables are written
    constexpr int RS = SB_NT / 128, NU = 16;   // rows per thread and pass
    const int m = tid & 127;
    const int64_t moff = (int64_t)b * s_b + (int64_t)min(m, Ms - 1) * s_m;
#pragma unroll 1
    for (int k0 = tid >> 7; k0 < SB_K; k0 += RS * NU) {
      double v[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int k = k0 + RS * u;
        const double x = ld_as_double<TS>(srow[k] + moff);
        v[u] = (k < Kt && m < Ms) ? x : 0.0;
      }
#pragma unroll
      for (int u = 0; u < NU; ++u) Ss[k0 + RS * u][m] = v[u];
    }
    __syncthreads();
  };

  // T operand of chunk c of item it: b[kk][j] = T[CD c + 4kk + lane/16][n0 + 16 WN wave + 16j + lane%16]
  auto load_T = [&](int it, int c, double (&bf)[KS][WN]) {
    const int b = it / tilesN, tn = it % tilesN;
    const int64_t boff = (int64_t)b * t_b;
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int n = min(tn * SB_TN + wave * 16 * WN + 16 * j + (lane & 15), Ns - 1);
      const int64_t noff = boff + n * t_n;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) bf[kk][j] = ld_as_double<TT>(trow[c * CD + 4 * kk + (lane >> 4)] + noff);
    }
  };

  int it = blockIdx.x;
  if (it >= nitems) return;
  int cur_b = it / tilesN;
  __syncthreads();   // row tables visible
  double bc[KS][WN], bn[KS][WN];
  load_T(it, 0, bc);   // in flight during the fill of S
  load_S(cur_b);
  while (true) {
    const int next = it + gridDim.x;
    doublex4 acc[NRB][WN];
#pragma unroll
    for (int i = 0; i < NRB; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[i][j] = doublex4{0, 0, 0, 0};
    for (int c = 0; c < nchunk; ++c) {
      // prefetch the next chunk: of this item, or the first of the next item
      const bool more_here = c + 1 < nchunk;
      if (more_here) load_T(it, c + 1, bn);
      else if (next < nitems) load_T(next, 0, bn);
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int k = c * CD + 4 * kk + (lane >> 4);
        double a[NRB];
#pragma unroll
        for (int i = 0; i < NRB; ++i) a[i] = Ss[k][16 * i + (lane & 15)];
#pragma unroll
        for (int i = 0; i < NRB; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bc[kk][j], acc[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
#pragma unroll
        for (int j = 0; j < WN; ++j) bc[kk][j] = bn[kk][j];
    }
    // epilogue: lane holds rows 16i + 4v + lane/16, column 16j + lane%16
    {
      const int b = it / tilesN, tn = it % tilesN;
      char* Cb = reinterpret_cast<char*>(D.C) + (int64_t)b * D.sCb * (tC == F64 ? 8 : 4);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int n = tn * SB_TN + wave * 16 * WN + 16 * j + (lane & 15);
#pragma unroll
        for (int i = 0; i < NRB; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = 16 * i + 4 * v + (lane >> 4);
            if (m < Ms && n < Ns) {
              const int64_t off = m * c_m + n * c_n;
              const double val = alpha * acc[i][j][v];
              if (tC == F64) gst(reinterpret_cast<double*>(Cb) + off, val);
              else gst(reinterpret_cast<float*>(Cb) + off, (float)val);
            }
          }
      }
    }
    if (next >= nitems) break;
    const int nb = next / tilesN;
    if (nb != cur_b && s_b != 0) {
      cur_b = nb;
      load_S(cur_b);
    }
    it = next;
  }
}

// The same product for reductions of 97 .. 128 (four 32-deep chunks per
// item), with a ring of four operand buffers: the loads of a chunk are issued
// two chunks before it is needed, and those of the next item's first three
// chunks before the item's results are stored.  The vector-memory counter
// counts loads and stores in issue order; here the first wait with a store
// ahead of it comes two chunks after the stores, which have drained by then.
// Every item runs the same straight-line sequence (past the last item the
// loads repeat its last chunk), so every wait count is fixed.
template <typename TS, typename TT, typename TC>
__global__ __launch_bounds__(512, 1) void gemm_sb_ring_kernel(const GemmDesc* __restrict__ descs, int swap) {
  constexpr int NT = 512;
  __shared__ double Ss[SB_K][SB_MP];
  __shared__ const char* trow[SB_K];
  __shared__ const char* srow[SB_K];

  const GemmDesc& D = descs[blockIdx.y];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int Ms = swap ? D.N : D.M;
  const int Ns = swap ? D.M : D.N;
  const int nseg = D.nseg > 0 ? D.nseg : 1;
  const int esS = sizeof(TS), esT = sizeof(TT);
  const int64_t s_m = (swap ? D.sBn : D.sAm) * esS;
  const int64_t t_n = (swap ? D.sAm : D.sBn) * esT;
  const int64_t s_b = (swap ? D.sBb : D.sAb) * esS;
  const int64_t t_b = (swap ? D.sAb : D.sBb) * esT;
  const int64_t c_m = swap ? D.sCn : D.sCm, c_n = swap ? D.sCm : D.sCn;
  int Kt = 0;
  for (int s = 0; s < nseg; ++s) Kt += D.nseg > 0 ? D.segK[s] : D.K;
  if (tid < SB_K) {
    const int k = min(tid, Kt - 1);
    int s = 0, kofs = 0;
    while (s + 1 < nseg && k >= kofs + (D.nseg > 0 ? D.segK[s] : D.K)) {
      kofs += D.nseg > 0 ? D.segK[s] : D.K;
      ++s;
    }
    const int kl = k - kofs;
    const char* Aseg = reinterpret_cast<const char*>(D.nseg > 0 ? D.segA[s] : D.A);
    const int64_t sAk = D.nseg > 0 ? D.segAk[s] : D.sAk;
    const int64_t boff = D.nseg > 0 ? D.segBoff[s] : 0;
    const char* Bb = reinterpret_cast<const char*>(D.B);
    if (!swap) {
      srow[tid] = Aseg + kl * sAk * esS;
      trow[tid] = Bb + (boff + kl * D.sBk) * esT;
    } else {
      srow[tid] = Bb + (boff + kl * D.sBk) * esS;
      trow[tid] = Aseg + kl * sAk * esT;
    }
  }
  const int tilesN = (Ns + SB_TN - 1) / SB_TN;
  const int nitems = tilesN * D.nbatch;
  const int it0 = blockIdx.x;
  if (it0 >= nitems) return;
  const int nq = (nitems - it0 + (int)gridDim.x - 1) / (int)gridDim.x;   // items of this workgroup

  // S into LDS as in gemm_sb_kernel: all loads of a thread in flight at once
  auto load_S = [&](int b) {
    __syncthreads();
    constexpr int RS = NT / 128, NU = 16;   // rows per thread and pass
    const int m = tid & 127;
    const int64_t moff = (int64_t)b * s_b + (int64_t)min(m, Ms - 1) * s_m;
#pragma unroll 1
    for (int k0 = tid >> 7; k0 < SB_K; k0 += RS * NU) {
      double v[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int k = k0 + RS * u;
        const double x = ld_as_double<TS>(srow[k] + moff);
        v[u] = (k < Kt && m < Ms) ? x : 0.0;
      }
#pragma unroll
      for (int u = 0; u < NU; ++u) Ss[k0 + RS * u][m] = v[u];
    }
    __syncthreads();
  };
  // chunk c (32 deep) of the q-th item of this workgroup, q clamped to the last
  auto load_T = [&](int q, int c, double (&bf)[8]) {
    const int it = it0 + min(q, nq - 1) * (int)gridDim.x;
    const int b = it / tilesN, tn = it % tilesN;
    const int n = min(tn * SB_TN + wave * 16 + (lane & 15), Ns - 1);
    const int64_t noff = (int64_t)b * t_b + n * t_n;
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) bf[kk] = ld_as_double<TT>(trow[32 * c + 4 * kk + (lane >> 4)] + noff);
  };
  // the scale is always loaded (from the descriptor itself without a device
  // factor) so that no load sits behind a branch
  const double av = gld(D.alpha_dev ? D.alpha_dev : &D.alpha);
  const double alpha = D.alpha_dev ? D.alpha * av : av;

  int cur_b = it0 / tilesN;
  __syncthreads();   // row tables visible
  double B0[8], B1[8], B2[8], B3[8];
  load_T(0, 0, B0);   // the first three chunks are in flight during the fill of S
  load_T(0, 1, B1);
  load_T(0, 2, B2);
  load_S(cur_b);
  doublex4 acc[8];
  auto chunk = [&](int c, const double (&bf)[8]) {
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 32 * c + 4 * kk + (lane >> 4);
      double a[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = Ss[k][16 * i + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bf[kk], acc[i], 0, 0, 0);
    }
  };
  for (int q = 0; q < nq; ++q) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = doublex4{0, 0, 0, 0};
    // each prefetch is issued after the chunk it follows: with three
    // buffers of eight loads and the 32 stores of an item at most 56 memory
    // operations are outstanding at any wait (the counter holds 63)
    chunk(0, B0);
    load_T(q, 3, B3);
    chunk(1, B1);
    load_T(q + 1, 0, B0);
    chunk(2, B2);
    load_T(q + 1, 1, B1);
    chunk(3, B3);
    load_T(q + 1, 2, B2);
    // epilogue: lane holds rows 16i + 4v + lane/16, column lane%16 of the wave's strip
    {
      const int it = it0 + q * (int)gridDim.x;
      const int b = it / tilesN, tn = it % tilesN;
      TC* Cb = reinterpret_cast<TC*>(D.C) + (int64_t)b * D.sCb;
      const int n = tn * SB_TN + wave * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * i + 4 * v + (lane >> 4);
          const bool in = m < Ms && n < Ns;
          TC* p = in ? Cb + (m * c_m + n * c_n) : reinterpret_cast<TC*>(&g_sb_sink[tid]);
          gst(p, (TC)(alpha * acc[i][v]));
        }
    }
    if (q + 1 < nq && s_b != 0) {
      const int nb = (it0 + (q + 1) * (int)gridDim.x) / tilesN;
      if (nb != cur_b) {
        cur_b = nb;
        load_S(cur_b);
      }
    }
  }
}

template <typename TS, typename TT, int CD>
void go_sb_rows(const GemmLaunch& g, dim3 grid, hipStream_t s) {
  // row blocks for the largest small operand of the launch
  if (g.sb_rows <= 32)
    hipLaunchKernelGGL((gemm_sb_kernel<TS, TT, 1, CD, 2>), grid, dim3(512), 0, s, g.descs, g.sb_swap, g.tC);
  else if (g.sb_rows <= 64)
    hipLaunchKernelGGL((gemm_sb_kernel<TS, TT, 1, CD, 4>), grid, dim3(512), 0, s, g.descs, g.sb_swap, g.tC);
  else if (g.sb_rows <= 96)
    hipLaunchKernelGGL((gemm_sb_kernel<TS, TT, 1, CD, 6>), grid, dim3(512), 0, s, g.descs, g.sb_swap, g.tC);
  else
    hipLaunchKernelGGL((gemm_sb_kernel<TS, TT, 1, CD, 8>), grid, dim3(512), 0, s, g.descs, g.sb_swap, g.tC);
}

template <typename TS, typename TT>
hipError_t go_sb(const GemmLaunch& g, hipStream_t s) {
  dim3 grid(g.sb_grid, g.ndesc, 1);
  if (g.sb_ring && g.tC == F64)
    hipLaunchKernelGGL((gemm_sb_ring_kernel<TS, TT, double>), grid, dim3(512), 0, s, g.descs, g.sb_swap);
  else if (g.sb_ring)
    hipLaunchKernelGGL((gemm_sb_ring_kernel<TS, TT, float>), grid, dim3(512), 0, s, g.descs, g.sb_swap);
  else if (g.sb_cd == 64)
    go_sb_rows<TS, TT, 64>(g, grid, s);
  else
    go_sb_rows<TS, TT, 32>(g, grid, s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_sb(const GemmLaunch& g, hipStream_t s) {
  // S is B when swapped, A otherwise; T the other one
  const int tS = g.sb_swap ? g.tB : g.tA, tT = g.sb_swap ? g.tA : g.tB;
  if (tS == F32 && tT == F32) return go_sb<float, float>(g, s);
  if (tS == F32) return go_sb<float, double>(g, s);
  if (tT == F32) return go_sb<double, float>(g, s);
  return go_sb<double, double>(g, s);
}

}  // namespace ht
