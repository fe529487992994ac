// Long reductions with a small result,
//   C[m][n] (+)= alpha * sum_k A[m][k] B[k][n],   m < M <= 128, n < N <= 128,
// split over k between workgroups that add their partial results atomically:
// the Gram matrices of both CholeskyQR2 sweeps (W^T W of the leaf frames and
// M1(B') M1(B')^T of the transfer tensors, Section 3.4) and the son Gramians
// of eqs. (acctransferSon1/2), reductions over 1e4 .. 1.6e4 terms.
//
// A workgroup owns the whole 128 x 128 result for its slice of k.  The slice
// moves through LDS in 16-deep chunks (double-buffered, next chunk prefetched
// into registers, one barrier per chunk), loaded along whichever index of
// each operand is contiguous.  Fragments are read as four consecutive k per
// lane: MFMA q of a 16-deep step then pairs k = 4j + q of A with the same k
// of B in lane group j, so the four products cover the chunk exactly, with A
// and B permuted alike.  When the result is symmetric (a Gram matrix, B = A^T
// of the same matrix, or a son Gramian, which inherits the symmetry of
// Bhat_t) only the 36 blocks of 16 x 16 on or above the diagonal are formed,
// each wave taking the nine blocks of block rows w and 7-w, and the
// off-diagonal blocks are added at both places.  A son Gramian whose operands
// are both contiguous along their row index stages its chunks k-major (a
// chunk row holds 128 consecutive rows): each load instruction then reads
// 512 contiguous bytes and each LDS write covers all banks once.
#include <type_traits>

#include "ht_internal.h"

namespace ht {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int RK_NT = 256;

template <typename TM> struct RkTraits;
template <> struct RkTraits<double> {
  using V = doublex4;
  static constexpr int PAD = 2;   // row stride 18 doubles = 144 B (16-B aligned fragments)
  __device__ static V mfma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // FP64 16x16x4: register v of lane l holds row 4v + l/16
  __device__ static int row(int v, int lane) { return 4 * v + (lane >> 4); }
};
template <> struct RkTraits<float> {
  using V = floatx4;
  static constexpr int PAD = 4;   // row stride 20 floats = 80 B
  __device__ static V mfma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // FP32 16x16x4: register v of lane l holds row 4(l/16) + v
  __device__ static int row(int v, int lane) { return 4 * (lane >> 4) + v; }
};

// MODE 0: full result; 1: Gram matrix (B = A^T, upper blocks); 2: separate B
// but a symmetric result (upper blocks, mirrored), as for the son Gramians
// PART: some result of the launch has at most 112 rows, and the block
// columns past a result are skipped (a run-time test the full-size launches do
// not carry).
template <typename TA, typename TB, typename TM, int MODE, int RK_KC, bool KM = false, bool PART = false>
__global__ __launch_bounds__(RK_NT, MODE != 0 ? 2 : 1) void gemm_rk_kernel(const GemmDesc* __restrict__ descs,
                                                                        int nsplit, int tC, int mode) {
  constexpr bool SYM = MODE != 0;      // upper blocks only
  constexpr bool SAMEB = MODE == 1;    // B fragments read from A
  constexpr int LU = RK_KC / 2;   // elements per thread per operand and chunk
  using Tr = RkTraits<TM>;
  using V = typename Tr::V;
  constexpr int LDK = RK_KC + Tr::PAD;
  __shared__ TM As[2][128][LDK];
  __shared__ TM Bs[SAMEB ? 1 : 2][SAMEB ? 1 : 128][LDK];
  // KM: both operands contiguous along their row index, staged k-major
  // (chunk row k holds 128 consecutive rows), written and read without
  // bank conflicts
  static_assert(!KM || (MODE == 2 && RK_KC * 128 <= 128 * LDK), "k-major staging");
  TM (*const Ak)[128] = reinterpret_cast<TM (*)[128]>(&As[0][0][0]);   // [buf * RK_KC + k][r]
  TM (*const Bk)[128] = reinterpret_cast<TM (*)[128]>(&Bs[0][0][0]);
  constexpr int KMB = (128 * LDK) / 128;   // k rows per buffer in the k-major view

  const GemmDesc& D = descs[blockIdx.y];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = D.M, N = D.N, K = D.K;
  const int cpb = (K + RK_KC - 1) / RK_KC;          // chunks per reduction block
  const int total = cpb * D.KB;
  const int per = (total + nsplit - 1) / nsplit;
  const int c0 = blockIdx.x * per, c1 = min(total, c0 + per);
  if (c0 >= c1) return;

  const bool a_kc = D.sAk == 1, b_kc = D.sBk == 1;
  const int nbk = (max(M, N) + 15) >> 4;   // 16 x 16 blocks along each side holding result rows
  const TA* Ab = reinterpret_cast<const TA*>(D.A);
  const TB* Bb = reinterpret_cast<const TB*>(D.B);
  const int msplit = D.msplit > 0 ? D.msplit : M;   // rows from here on lie a2off further
  // offset of element (r, k) of A in chunk segment kb (row and k clamped, so
  // every load is in bounds; entries past K are masked when stashed)
  auto aoff = [&](int kb, int r, int k) -> int64_t {
    const int rr = min(r, M - 1);
    return (int64_t)kb * D.sAkb + (int64_t)rr * D.sAm + (rr >= msplit ? D.a2off : 0) +
           (int64_t)min(k, K - 1) * D.sAk;
  };

  // loader coordinates: along k (thread t: k t % KC of rows t / KC + (256 / KC) u,
  // so that KC consecutive lanes read one row's chunk and write one LDS row)
  // or along the row index (thread t: k t/(128/LU), LU rows from (t%(128/LU))*LU).
  // The prefetched values stay raw (operand type, unmasked) until the chunk
  // is stashed after the current chunk's products, so nothing before those
  // products waits for them.
  constexpr int RG = 128 / LU;
  constexpr int KR = 256 / RK_KC;   // rows per pass of the k-contiguous loader
  TA ra[LU];
  TB rb[LU];
  auto kof = [&](int u) -> int {   // k within the chunk of this thread's value u
    if constexpr (KM) return (tid >> 7) * LU + u;
    return a_kc ? tid % RK_KC : tid / RG;
  };
  auto kofb = [&](int u) -> int {
    if constexpr (KM) return (tid >> 7) * LU + u;
    return b_kc ? tid % RK_KC : tid / RG;
  };
  auto load = [&](int c) {
    const int kb = c / cpb, k0 = (c % cpb) * RK_KC;
    const TB* Bg = Bb + (int64_t)kb * D.sBkb;
    if constexpr (KM) {   // thread t: row t % 128, k from (t / 128) * LU
#pragma unroll
      for (int u = 0; u < LU; ++u) ra[u] = gld(&Ab[aoff(kb, tid & 127, k0 + kof(u))]);
#pragma unroll
      for (int u = 0; u < LU; ++u) {
        const int n = tid & 127, k = k0 + kofb(u);
        rb[u] = gld(&Bg[(int64_t)min(k, K - 1) * D.sBk + (int64_t)min(n, N - 1) * D.sBn]);
      }
      return;
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int r = a_kc ? tid / RK_KC + KR * u : (tid % RG) * LU + u;
      ra[u] = gld(&Ab[aoff(kb, r, k0 + kof(u))]);
    }
    if (!SAMEB) {
#pragma unroll
      for (int u = 0; u < LU; ++u) {
        const int n = b_kc ? tid / RK_KC + KR * u : (tid % RG) * LU + u;
        const int k = k0 + kofb(u);
        rb[u] = gld(&Bg[(int64_t)min(k, K - 1) * D.sBk + (int64_t)min(n, N - 1) * D.sBn]);
      }
    }
  };
  // converted to the math type and masked past K as they go to LDS
  auto stash = [&](int buf, int c) {
    const int k0 = (c % cpb) * RK_KC;
    if constexpr (KM) {
#pragma unroll
      for (int u = 0; u < LU; ++u) {
        Ak[buf * KMB + (tid >> 7) * LU + u][tid & 127] = (TM)ra[u] * (TM)(k0 + kof(u) < K);
        Bk[buf * KMB + (tid >> 7) * LU + u][tid & 127] = (TM)rb[u] * (TM)(k0 + kofb(u) < K);
      }
      return;
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int r = a_kc ? tid / RK_KC + KR * u : (tid % RG) * LU + u;
      As[buf][r][kof(u)] = (TM)ra[u] * (TM)(k0 + kof(u) < K);
    }
    if (!SAMEB) {
#pragma unroll
      for (int u = 0; u < LU; ++u) {
        const int n = b_kc ? tid / RK_KC + KR * u : (tid % RG) * LU + u;
        Bs[buf][n][kofb(u)] = (TM)rb[u] * (TM)(k0 + kofb(u) < K);
      }
    }
  };

  // result writes (scale read after the reduction, in each epilogue)
  auto put = [&](int m, int n, double val) {
    const int64_t off = (int64_t)m * D.sCm + (int64_t)n * D.sCn;
    if (tC == F64) {
      double* p = reinterpret_cast<double*>(D.C) + off;
      if (mode == GEMM_ATOMIC) gatomic_add(p, val); else gst(p, val);
    } else {
      float* p = reinterpret_cast<float*>(D.C) + off;
      if (mode == GEMM_ATOMIC) gatomic_add(p, (float)val); else gst(p, (float)val);
    }
  };
  auto scale = [&]() {
    double alpha = D.alpha;
    if (D.alpha_dev) alpha *= gld(D.alpha_dev);
    return alpha;
  };

  load(c0);
  stash(0, c0);
  __syncthreads();
  int buf = 0;
  if constexpr (SAMEB) {
    // Gram matrix: block rows w and 7-w against the block columns right of
    // them; the column fragments of one step are read once and serve both
    // rows.  The loop is compiled once per wave, so that each wave's block
    // set is fixed at compile time and its products run without branches.
    auto gram = [&](auto wc) {
      constexpr int W = decltype(wc)::value;
      V acc[2][8];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = V{0, 0, 0, 0};
      for (int c = c0; c < c1; ++c) {
        const bool more = c + 1 < c1;
        if (more) load(c + 1);
#pragma unroll
        for (int st = 0; st < RK_KC / 16; ++st) {
          const int kq = 16 * st + 4 * (lane >> 4);
#pragma unroll
          for (int hq = 0; hq < 2; ++hq) {
            TM fa[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
              const TM* p = &As[buf][16 * (i == 0 ? W : 7 - W) + (lane & 15)][kq + 2 * hq];
              fa[i][0] = p[0];
              fa[i][1] = p[1];
            }
            // block columns left of both rows are skipped; a column's two
            // fragments are read just before its products
#pragma unroll
            for (int j = W; j < 8; ++j) {
              if (PART && j >= nbk) continue;   // block column past the result (its row is at most j)
              const TM* p = &As[buf][16 * j + (lane & 15)][kq + 2 * hq];
              const TM fb0 = p[0], fb1 = p[1];
#pragma unroll
              for (int i = 0; i < 2; ++i)
                if (j >= (i == 0 ? W : 7 - W)) acc[i][j] = Tr::mfma(fa[i][0], fb0, acc[i][j]);
#pragma unroll
              for (int i = 0; i < 2; ++i)
                if (j >= (i == 0 ? W : 7 - W)) acc[i][j] = Tr::mfma(fa[i][1], fb1, acc[i][j]);
            }
          }
        }
        if (more) stash(buf ^ 1, c + 1);
        __syncthreads();
        buf ^= 1;
      }
      const double alpha = scale();
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = (i == 0 ? W : 7 - W); j < 8; ++j) {
          const int rbk = i == 0 ? W : 7 - W;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = 16 * rbk + Tr::row(v, lane), n = 16 * j + (lane & 15);
            if (m < M && n < N) {
              const double val = alpha * (double)acc[i][j][v];
              put(m, n, val);
              if (j != rbk) put(n, m, val);
            }
          }
        }
    };
    switch (__builtin_amdgcn_readfirstlane(wave)) {
      case 0: gram(std::integral_constant<int, 0>{}); break;
      case 1: gram(std::integral_constant<int, 1>{}); break;
      case 2: gram(std::integral_constant<int, 2>{}); break;
      case 3: gram(std::integral_constant<int, 3>{}); break;
      default: __builtin_unreachable();
    }
  } else if constexpr (SYM) {
    // symmetric result of two operands: the wave's nine blocks, row block w
    // against columns w..7, then row block 7-w against columns 7-w..7 (36
    // upper blocks over four waves); exactly nine accumulators, so two
    // workgroups fit a CU
    const int nfirst = 8 - wave;
    auto bcol = [&](int bl) { return bl < nfirst ? wave + bl : (7 - wave) + (bl - nfirst); };
    V acc[9];
#pragma unroll
    for (int bl = 0; bl < 9; ++bl) acc[bl] = V{0, 0, 0, 0};
    for (int c = c0; c < c1; ++c) {
      const bool more = c + 1 < c1;
      if (more) load(c + 1);
#pragma unroll
      for (int st = 0; st < RK_KC / 16; ++st) {
        const int kq = 16 * st + 4 * (lane >> 4);
#pragma unroll
        for (int hq = 0; hq < 2; ++hq) {
          TM fa0[2], fa1[2];
          if constexpr (KM) {
            const int kr = buf * KMB + kq + 2 * hq;
            fa0[0] = Ak[kr][16 * wave + (lane & 15)];
            fa0[1] = Ak[kr + 1][16 * wave + (lane & 15)];
            fa1[0] = Ak[kr][16 * (7 - wave) + (lane & 15)];
            fa1[1] = Ak[kr + 1][16 * (7 - wave) + (lane & 15)];
          } else {
            const TM* pa0 = &As[buf][16 * wave + (lane & 15)][kq + 2 * hq];
            const TM* pa1 = &As[buf][16 * (7 - wave) + (lane & 15)][kq + 2 * hq];
            fa0[0] = pa0[0]; fa0[1] = pa0[1]; fa1[0] = pa1[0]; fa1[1] = pa1[1];
          }
#pragma unroll
          for (int bl = 0; bl < 9; ++bl) {
            const int col = bcol(bl);
            TM fb0, fb1;
            if constexpr (KM) {
              const int kr = buf * KMB + kq + 2 * hq;
              fb0 = Bk[kr][16 * col + (lane & 15)];
              fb1 = Bk[kr + 1][16 * col + (lane & 15)];
            } else {
              const TM* pb = SAMEB ? &As[buf][16 * col + (lane & 15)][kq + 2 * hq]
                                   : &Bs[buf][16 * col + (lane & 15)][kq + 2 * hq];
              fb0 = pb[0];
              fb1 = pb[1];
            }
            const bool first = bl < nfirst;
            if (!PART || col < nbk) {   // a block column past the result (its row is at most col) is skipped
              acc[bl] = Tr::mfma(first ? fa0[0] : fa1[0], fb0, acc[bl]);
              acc[bl] = Tr::mfma(first ? fa0[1] : fa1[1], fb1, acc[bl]);
            }
          }
        }
      }
      if (more) stash(buf ^ 1, c + 1);
      __syncthreads();
      buf ^= 1;
    }
    const double alpha = scale();
#pragma unroll
    for (int bl = 0; bl < 9; ++bl) {
      const int rbk = bl < nfirst ? wave : 7 - wave, cbk = bcol(bl);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * rbk + Tr::row(v, lane), n = 16 * cbk + (lane & 15);
        if (m < M && n < N) {
          const double val = alpha * (double)acc[bl][v];
          put(m, n, val);
          if (cbk != rbk) put(n, m, val);
        }
      }
    }
  } else {
    // full result: wave w owns block rows 4(w/2) .. +3 and columns 4(w%2) .. +3
    V acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = V{0, 0, 0, 0};
    for (int c = c0; c < c1; ++c) {
      const bool more = c + 1 < c1;
      if (more) load(c + 1);
#pragma unroll
      for (int st = 0; st < RK_KC / 16; ++st) {
        const int kq = 16 * st + 4 * (lane >> 4);
#pragma unroll
        for (int hq = 0; hq < 2; ++hq) {
          TM fa[4][2], fb[4][2];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const TM* p = &As[buf][16 * (4 * (wave >> 1) + i) + (lane & 15)][kq + 2 * hq];
            fa[i][0] = p[0];
            fa[i][1] = p[1];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const TM* p = &Bs[buf][16 * (4 * (wave & 1) + j) + (lane & 15)][kq + 2 * hq];
            fb[j][0] = p[0];
            fb[j][1] = p[1];
          }
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j) acc[i][j] = Tr::mfma(fa[i][q], fb[j][q], acc[i][j]);
        }
      }
      if (more) stash(buf ^ 1, c + 1);
      __syncthreads();
      buf ^= 1;
    }
    const double alpha = scale();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * (4 * (wave >> 1) + i) + Tr::row(v, lane), n = 16 * (4 * (wave & 1) + j) + (lane & 15);
          if (m < M && n < N) put(m, n, alpha * (double)acc[i][j][v]);
        }
  }
}

template <typename TA, typename TB, typename TM, bool PART>
void go_rk_part(const GemmLaunch& g, dim3 grid, hipStream_t s) {
  if (g.rk_sym == 1)
    hipLaunchKernelGGL((gemm_rk_kernel<TA, TB, TM, 1, 32, false, PART>), grid, dim3(RK_NT), 0, s, g.descs, g.rk_split,
                       g.tC, g.mode);
  else if (!g.a_kcontig && !g.b_kcontig)
    hipLaunchKernelGGL((gemm_rk_kernel<TA, TB, TM, 2, 16, true, PART>), grid, dim3(RK_NT), 0, s, g.descs, g.rk_split,
                       g.tC, g.mode);
  else
    hipLaunchKernelGGL((gemm_rk_kernel<TA, TB, TM, 2, 16, false, PART>), grid, dim3(RK_NT), 0, s, g.descs, g.rk_split,
                       g.tC, g.mode);
}

template <typename TA, typename TB, typename TM>
hipError_t go_rk(const GemmLaunch& g, hipStream_t s) {
  dim3 grid(g.rk_split, g.ndesc, 1);
  if (g.rk_sym == 0)
    hipLaunchKernelGGL((gemm_rk_kernel<TA, TB, TM, 0, 16>), grid, dim3(RK_NT), 0, s, g.descs, g.rk_split, g.tC,
                       g.mode);
  else if (g.rk_part)
    go_rk_part<TA, TB, TM, true>(g, grid, s);
  else
    go_rk_part<TA, TB, TM, false>(g, grid, s);
  return hipGetLastError();
}

template <typename TM>
hipError_t go_rk_types(const GemmLaunch& g, hipStream_t s) {
  const bool a32 = g.tA == F32, b32 = g.tB == F32;
  if (a32 && b32) return go_rk<float, float, TM>(g, s);
  if (a32) return go_rk<float, double, TM>(g, s);
  if (b32) return go_rk<double, float, TM>(g, s);
  return go_rk<double, double, TM>(g, s);
}

}  // namespace

hipError_t launch_gemm_rk(const GemmLaunch& g, hipStream_t s) {
  return g.math == MATH_F32 ? go_rk_types<float>(g, s) : go_rk_types<double>(g, s);
}

}  // namespace ht
