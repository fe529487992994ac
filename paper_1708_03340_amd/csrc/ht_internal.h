// Internal declarations of the HT hierarchical-SVD library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace ht {

// Largest sum rank the LDS-resident small dense kernels accept.
constexpr int KMAX = 128;
// Segments of a segmented reduction (one per summand of a lazy sum).
constexpr int MAX_SEG = 8;

// Eigensolver scratch layout (eig.hip), in doubles from the node's scratch
// pointer: the Householder reflectors (K x K) and their tau (K), then the
// eigenvector blocks of the divide-and-conquer merges.  The tridiagonal of
// order K is cut in halves down to single rows: at depth t block b is
// [floor(b K / 2^t), floor((b+1) K / 2^t)), at most ceil(K / 2^t) rows, and
// merges its two halves.  The merges of depth t write their m x m eigenvector
// blocks into a region of K ceil(K / 2^t) + 8 doubles of their own (block
// [lo, hi) at lo * ceil(K / 2^t)), so no address is written twice in a launch.
__host__ __device__ inline int dc_depths(int K) {          // ceil(log2 K), 0 for K <= 1
  int t = 0;
  while ((1 << t) < K) ++t;
  return t;
}
__host__ __device__ inline int64_t dc_region_doubles(int K, int t) {
  return (int64_t)K * (((K - 1) >> t) + 1) + 8;
}
__host__ __device__ inline int64_t eig_reflector_doubles(int K) { return (int64_t)K * K + K + 64; }
__host__ __device__ inline int64_t eig_scratch_doubles(int K) {
  int64_t s = eig_reflector_doubles(K);
  for (int t = 0; t < dc_depths(K); ++t) s += dc_region_doubles(K, t);
  return s;
}

// Element types of GEMM operands / results.
enum DType : int { F64 = 0, F32 = 1 };

// One strided (batched) GEMM problem: C(m,n) (op)= alpha * sum_r A(m,r) B(r,n).
//   A(m,k) = A[m*sAm + k*sAk], B(k,n) = B[k*sBk + n*sBn], C(m,n) = C[m*sCm + n*sCn].
// The reduction index r runs over KB blocks of K (block kb shifts A by kb*sAkb and
// B by kb*sBkb) or, if nseg > 0, over nseg segments with their own A base,
// B offset and length.  nbatch independent problems differ by sAb/sBb/sCb.
struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  int64_t sAm, sAk, sBk, sBn, sCm, sCn;
  int64_t sAb, sBb, sCb;
  int64_t sAkb, sBkb;
  int32_t M, N, K, KB;
  int32_t nbatch, nseg;
  const void* segA[MAX_SEG];
  int64_t segBoff[MAX_SEG];
  int32_t segK[MAX_SEG];
  int64_t segAk[MAX_SEG];   // per-segment k-stride of A
  // Khatri-Rao operand (entry evaluation, eq. (transfermult)): if kr != 0,
  // A(m,k) = krY1[m*krld1 + k / krK2] * krY2[m*krld2 + k % krK2] (float64 rows).
  int32_t kr, krK2;
  const double* krY1;
  const double* krY2;
  int64_t krld1, krld2;
  double alpha;
  const double* alpha_dev;  // if set, alpha is multiplied by *alpha_dev
  // Rows m >= msplit of A (msplit > 0) lie a2off elements further on, at
  // A + m*sAm + a2off: the Gram matrix of two frames with the same row
  // stride side by side, each in its own buffer.  Split-K Gram launches only.
  int64_t a2off;
  int32_t msplit;
};

// How a GEMM writes C.
enum GemmMode : int { GEMM_STORE = 0, GEMM_ATOMIC = 1 };
// Which matrix cores: FP32 MFMA (float accumulate) or FP64 MFMA.
enum GemmMath : int { MATH_F32 = 0, MATH_F64 = 1 };

struct GemmLaunch {
  int tA, tB, tC;          // DType of A, B, C
  int math;                // GemmMath
  int mode;                // GemmMode
  bool a_kcontig;          // sAk == 1 (else sAm == 1)
  bool b_kcontig;          // sBk == 1 (else sBn == 1)
  int splitk;              // blocks along the reduction (GEMM_ATOMIC if > 1)
  bool acc64;              // MATH_F32 only: float64 accumulation across k-slabs
  bool big;                // MATH_F64 only: 128 x 128 tiles
  bool sb;                 // MATH_F64, GEMM_STORE: small operand in LDS, the other streamed
  bool sb_swap;            //   small operand is B (A streamed along M)
  int sb_grid;             //   workgroups per descriptor
  int sb_wn;               //   16-column MFMA blocks per wave (2: 4 waves, else 8 waves)
  int sb_cd;               //   chunk depth along k: 64 (reduction a multiple of 64) or 32
  bool sb_ring;            //   every reduction is 97 .. 128: four-buffer ring kernel
  int sb_rows;             //   largest row count of the small operand (other kernels: 128)
  bool rk_part;            //   split-K: some result has at most 112 rows (skip past it)
  bool rk;                 // M, N <= 128, long reduction split over workgroups
  int rk_sym;              //   1: B is A^T of the same matrix; 2: symmetric result (upper blocks only)
  int rk_split;            //   workgroups per descriptor along the reduction
  int rk_kc;               //   k per LDS chunk (32 for rk_sym == 1, else 16)
  int ndesc, maxbatch, maxtiles;
  const GemmDesc* descs;   // device pointer
};

// Global-memory accesses made through the global address space.  Pointers
// read from argument tables are generic, and generic (flat) loads also count
// against the LDS wait counter: every wait for an LDS operand would then also
// wait for the HBM loads in flight.
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
__device__ __forceinline__ void gatomic_add(double* p, double v) {
  __builtin_amdgcn_global_atomic_fadd_f64((__attribute__((address_space(1))) double*)p, v);
}
__device__ __forceinline__ void gatomic_add(float* p, float v) {
  __builtin_amdgcn_global_atomic_fadd_f32((__attribute__((address_space(1))) float*)p, v);
}

hipError_t launch_gemm(const GemmLaunch& g, hipStream_t stream);
hipError_t launch_gemm_sb(const GemmLaunch& g, hipStream_t stream);
hipError_t launch_gemm_rk(const GemmLaunch& g, hipStream_t stream);

// ---------------------------------------------------------------- small dense kernels
// Per-node argument block of the small dense kernels (device-resident table).
struct SmallArgs {
  int32_t K;               // matrix order
  int32_t node;            // preorder node id
  int32_t rcap;            // projection width (output rank bound)
  int32_t rfix;            // fixed rank (>0) or 0 = read from rank_dev
  double* G;               // K x K Gram (input)
  double* G2;              // K x K second-sweep Gram
  double* R1;              // K x K first-sweep factor
  double* Ri1;             // K x K inverse of the first-sweep factor
  double* R;               // K x K upper factor R2 R1 (output, normalised by 2^-e)
  double* Ri;              // K x K inverse of the unnormalised factor
  double tol_rel;          // pivot tolerance relative to the largest diagonal entry
  double shift_rel;        // first sweep: diagonal shift relative to trace(G)
  void* Rf;                // K x K copy of R in the forward-product type
  int32_t rf_type;         // DType of Rf
  int32_t clamp_only;      // 1: first sweep (clamp tiny pivots), 0: final
  double* Q;               // K x K eigenvectors (columns, descending)
  double* lam;             // K eigenvalues (descending, >= 0)
  double* Qm;              // K x rcap masked leading eigenvectors
  void* QmT;               // rcap x K transpose in the forward type
  int32_t* rank_dev;       // rank of this node (device)
  double* sigma_out;       // optional: 128 slots for sigma / ||A||
  double* scratch;         // eigensolver scratch, eig_scratch_doubles(K)
  double* Bh;              // K x K Gramian (eigensolver input)
  struct GlobalState* st;  // state of the tensor this node belongs to (NULL: the launch's)
};

struct GlobalState {       // device-resident per-call scalars
  long long log2_scale;    // running scale exponent
  unsigned int flags;
  int pad;
  double alpha_gram;       // 2^(-2 e_D)
  long long e_D;           // binary exponent of ||B_D||_F
  double norm2_units;      // ||A||^2 in Gramian units (trace of Bhat_t1)
  double thr;              // tolerance threshold in Gramian units
  double alpha_root;       // 2^(-e_D): the truncated root is written in these units
};

// One tensor's scalars for the state kernels; a launch takes an array of
// them, one per tensor of a batch.
struct StateRec {
  GlobalState* st;
  long long scale0;        // set_state: initial binary exponent of the tensor
  const double* BD;        // root_norm: root matrix K1 x K2, row-major
  int32_t K1, K2;
  long long* out_scale;    // write_scale targets (each may be NULL)
  unsigned int* flags;
  int32_t* root_rank;
  int32_t add_eD;          // write_scale: add the root exponent e_D
  int32_t a0, na;          // rank selection: the tensor's nodes are args[a0 .. a0+na)
  int32_t d, mode, rel, t1, t2, pad;   // order, rank mode, relative eps, sons of the root
  double eps;
};
struct FillRec { void* p; size_t bytes; };   // zero p[0 .. bytes), bytes a multiple of 4
// dst[i*d0 + j*d1 + k*d2] = alpha * src[i*s0 + j*s1 + k*s2] over n0 x n1 x n2
struct CopyRec {
  const void* src;
  void* dst;
  int32_t tsrc, tdst;
  int64_t n0, n1, n2, s0, s1, s2, d0, d1, d2;
  double alpha;
};

// Power-of-two bookkeeping of the inner product (Definition (phi)) and the
// norm of an orthogonalised tensor (the Frobenius norm of its root matrix).
//   mode 0: e = binary exponent of max |P[i]|; P <- P 2^-e;
//           *E = e + (E1 ? *E1 : 0) + (E2 ? *E2 : 0).
//   mode 1: like mode 0, then *out_val = P[0] and
//           *out_log2 = *E + add + (add_dev ? *add_dev : 0) (P is 1 x 1).
//   mode 2: v = ||P||_F (over n entries); *out_val = v 2^-e with e the
//           exponent of v, *out_log2 = e + add + (add_dev ? *add_dev : 0).
// A non-finite entry sets bit 1 of *flags (if flags is not NULL).
struct PhiRec {
  double* P;
  int64_t n;
  long long* E;
  const long long* E1;
  const long long* E2;
  double* out_val;
  long long* out_log2;
  const long long* add_dev;
  long long add;
  unsigned int* flags;
  int32_t mode, pad;
};
hipError_t launch_phi_scale(const PhiRec* r, int n, hipStream_t s);

// Kronecker product of two transfer tensors (Lemma (operator)):
// F[(p,i)][(q,j)][(r,l)] = H[p][q][r] * B[i][j][l], the first factor's index
// slowest; H is P x Q x R, B is I x J x L, all row-major (a root matrix has
// P = I = 1).
struct KronRec {
  const void* H;
  const void* B;
  void* F;
  int32_t tH, tB, tF;
  int32_t P, Q, R, I, J, L;
  int32_t pad;
};
hipError_t launch_kron(const KronRec* r, int n, int64_t max_elems, int64_t max_a, hipStream_t s);

hipError_t launch_fill(const FillRec* r, int n, size_t max_bytes, hipStream_t s);
hipError_t launch_set_state(const StateRec* r, int n, hipStream_t s);
hipError_t launch_chol(const SmallArgs* args, int n, int sweep, hipStream_t s, GlobalState* st);
// max_k: the largest K among the args (picks the instantiation)
hipError_t launch_eig(const SmallArgs* args, int n, int max_k, hipStream_t s, GlobalState* st);
hipError_t launch_rank_select(const SmallArgs* args, const StateRec* r, int n, hipStream_t s);
hipError_t launch_proj_prep(const SmallArgs* args, int n, const GlobalState* st, hipStream_t s);
hipError_t launch_root_norm(const StateRec* r, int n, hipStream_t s);
hipError_t launch_write_scale(const StateRec* r, int n, hipStream_t s);
hipError_t launch_copy3(const CopyRec* r, int n, int64_t max_elems, hipStream_t s);
hipError_t launch_sigma_from_lam(const SmallArgs* args, int n, double* const* sigma_ptrs,
                                 hipStream_t s);

// ---------------------------------------------------------------- entries (Section 3.1)
struct EntryNode {
  int32_t k;               // rank of the node (row length)
  int32_t mode;            // leaves: 0-based mode
  int32_t tdtype;          // DType of the leaf frame
  int32_t pad;
  const void* U;           // leaves: column-major frame
  int64_t ld;              // leaves: leading dimension
  double* rows;            // m x k rows of this node (normalised in place)
  int32_t* expo;           // m binary exponents of this node
  const int32_t* expo1;    // inner: son exponents (added)
  const int32_t* expo2;
};
// leaves: rows[i][:] = U[idx[i][mode], :]; then every node: rows[i] /= 2^e_i.
hipError_t launch_entry_gather(const EntryNode* nodes, int n, int64_t m, const int32_t* idx, int d,
                               int maxk, hipStream_t s);
hipError_t launch_entry_normalize(const EntryNode* nodes, int n, int64_t m, int maxk, hipStream_t s);
// out[i] = rows_root[i] * 2^(expo_root[i] + log2_scale)
hipError_t launch_entry_finish(const double* vals, const int32_t* expo, int64_t m, long long log2_scale,
                               double* out, hipStream_t s);

// ---------------------------------------------------------------- tree (eq. (balanced))
struct Tree {
  int d = 0, nn = 0;
  std::vector<int> parent, son1, son2, lo, hi, depth, height, leaf_node;
  explicit Tree(int d_);
  bool is_leaf(int t) const { return son1[t] < 0; }
  int mode(int t) const { return lo[t]; }
  int max_depth() const;
};

}  // namespace ht
