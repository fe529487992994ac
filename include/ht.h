/*
 * ht.h -- C ABI of the MI355X (gfx950) hierarchical-SVD library for tensors in
 * the Hierarchical Tucker (HT) format.
 *
 * Method: Grasedyck & Loebbert, "Distributed Hierarchical SVD in the
 * Hierarchical Tucker Format".  Section numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Tree.      The balanced dimension tree of Section 2, eq. (balanced): node
 *            {mu..nu} has the sons {mu..floor((mu+nu-1)/2)} and the rest.
 *            Nodes are numbered in preorder (root = 0, then the whole first
 *            subtree, then the second); ht_tree() returns the numbering.
 * Tensor.    An ht_desc is a NON-OWNING view of one HT tensor (Section 2.1):
 *            leaf frames U_mu (column-major n_mu x k_mu, leading dimension
 *            leaf_ld[mu] >= n_mu), inner transfer tensors B_t (row-major
 *            [k_t][k_s1][k_s2], eq. (transfer)) and the root matrix B_D
 *            (row-major [k_t1][k_t2], always float64).  The represented
 *            tensor is 2^log2_scale times the tensor the data spells out.
 *            The caller owns every buffer; all data pointers are DEVICE
 *            pointers on the context's device, all arrays of pointers, sizes
 *            and ranks are HOST arrays read during the call only.
 * Streams.   Every call only enqueues work on `stream` (a hipStream_t, NULL =
 *            default stream) and returns; results are ready when the stream
 *            is.  Launch tables for a new combination of buffers are uploaded
 *            with one synchronous copy; repeating a call with the same
 *            buffers and shapes reuses them and makes no host synchronisation.
 * Threads.   A context may be shared by several host threads.  Each call
 *            holds the context's lock while it looks up or uploads its launch
 *            tables and enqueues, so launches of two calls never interleave
 *            and no table is freed while a call still has to enqueue from it.
 *            Calls on different streams that share a workspace or output
 *            buffers race on the device; the caller orders them (one stream,
 *            or events).
 * Errors.   Argument and shape errors are found on the host before anything
 *            is enqueued and returned as an ht_status; ht_last_error() gives
 *            a human-readable reason (per thread).  Numerical events (a
 *            rank-deficient frame met by the Cholesky step, a non-finite
 *            value, a tolerance not met under max_rank) are reported in the
 *            device `flags` word and never abort the call.
 * Sizes.     The *_workspace() queries are host-only and accept ctx == NULL;
 *            descriptors passed to them may have NULL data pointers.
 * Limits.    Sum ranks K_t <= 128 at every node (the small dense kernels keep
 *            a K x K float64 matrix in LDS); d >= 2; n_mu >= 1.
 */
#ifndef HT_H
#define HT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HT_OK = 0,
  HT_EINVAL = 1,        /* bad argument (NULL pointer, d < 2, bad mode, ...) */
  HT_ESHAPE = 2,        /* inconsistent shapes or ranks between descriptors */
  HT_EWORKSPACE = 3,    /* workspace too small or misaligned (256 B) */
  HT_EDEVICE = 4,       /* a HIP runtime call failed */
  HT_EUNSUPPORTED = 5   /* outside the limits above */
} ht_status;

typedef enum { HT_F64 = 0, HT_F32 = 1 } ht_dtype;

/* HT_PREC_FP64: every product in float64 on the FP64 matrix cores.
 * HT_PREC_MIXED: the first CholeskyQR2 sweep (the Gram matrices of the leaf
 *   frames and of M_{2,3} of every transfer tensor) may run on the FP32 matrix
 *   cores with float32 accumulation; the float64 second sweep removes its
 *   error.  Where the float64 split-K Gram kernel takes the shape (orders
 *   65..128; at the leaves, two summands whose frames share a row stride) it is
 *   used instead, being as fast.  Cholesky factors, inverses, the R-factor
 *   contractions, the orthogonal factors, the Gramian pass, the eigensolves and
 *   the projections are float64 (float32 there costs ~1e-6 relative error at
 *   d = 64). */
typedef enum { HT_PREC_FP64 = 0, HT_PREC_MIXED = 1 } ht_precision;

/* Truncation rank rule (Section 3.3 "for prescribed ranks or for prescribed
 * accuracy"):
 *   HT_RANK_FIXED: r_t = min(ranks[t], K_t).
 *   HT_RANK_TOL:   r_t = min{ r >= 1 : sum_{i>r} sigma_{t,i}^2 <= eps_abs^2/(2d-3) },
 *                  capped by max_rank (if > 0) and K_t; eps_abs = eps*||A|| if
 *                  eps_relative else eps.  The two sons of the root share the
 *                  rank computed at the first son. */
typedef enum { HT_RANK_FIXED = 0, HT_RANK_TOL = 1 } ht_rank_mode;

/* flags word bits (device uint32) */
#define HT_FLAG_RANK_DEFICIENT 1u   /* a Cholesky pivot vanished: that direction was dropped */
#define HT_FLAG_NONFINITE      2u   /* a NaN or Inf was met */
#define HT_FLAG_CAPPED         4u   /* max_rank stopped a node before eps was met */
#define HT_FLAG_NOCONV         8u   /* an eigenvalue of a Gramian was not resolved to working
                                       precision by the eigensolver's iteration limit; its
                                       eigenpair is used as it stands */
/* bits 8-15 of the flags word: the largest number of iterations any single
 * eigenvalue of any node's eigensolve needed (diagnostic, capped at 255) */

typedef struct ht_context ht_context;

typedef struct {
  int32_t d;                  /* number of modes, >= 2 */
  const int64_t* n;           /* [d]     mode sizes n_mu */
  const int32_t* rank;        /* [2d-1]  ranks k_t in preorder; rank[0] is ignored (k_D = 1) */
  int32_t frame_dtype;        /* ht_dtype of all leaf frames */
  int32_t transfer_dtype;     /* ht_dtype of all inner transfer tensors (the root is float64) */
  void* const* leaf;          /* [d]     U_mu, column-major n_mu x k_mu */
  const int64_t* leaf_ld;     /* [d]     leading dimensions, >= n_mu */
  void* const* transfer;      /* [2d-1]  B_t in preorder; entries of leaves are ignored */
  int64_t log2_scale;         /* tensor = 2^log2_scale * (stored tensor) */
} ht_desc;

typedef struct {
  int32_t mode;               /* ht_rank_mode */
  const int32_t* ranks;       /* [2d-1] host, HT_RANK_FIXED only */
  double eps;                 /* HT_RANK_TOL only, >= 0 */
  int32_t eps_relative;       /* HT_RANK_TOL: 1 = relative to ||A||, 0 = absolute */
  int32_t max_rank;           /* HT_RANK_TOL: rank cap, <= 0 for none */
  int32_t precision;          /* ht_precision */
} ht_trunc_opts;

/* ---------------------------------------------------------------- context */
/* Creates a context bound to HIP device `device` (its caches: launch tables).
 * Errors: HT_EINVAL (out == NULL), HT_EDEVICE (no such device). */
ht_status ht_create_context(int device, ht_context** out);
void ht_destroy_context(ht_context* ctx);
const char* ht_status_string(ht_status s);
const char* ht_last_error(void);
int32_t ht_version(void);

/* Tree of eq. (balanced) for dimension d, preorder numbering.  Every output
 * is a host array of 2d-1 int32 (any may be NULL): parent (-1 at the root),
 * son1/son2 (-1 at leaves), lo/hi (first/last 0-based mode of the node),
 * depth (root 0), height (leaves 0).  Errors: HT_EINVAL for d < 2. */
ht_status ht_tree(int32_t d, int32_t* parent, int32_t* son1, int32_t* son2,
                  int32_t* lo, int32_t* hi, int32_t* depth, int32_t* height);

/* ---------------------------------------------------------------- sum
 * S = alpha*A + beta*C by Lemma (sum), Section 3.5: S's leaf frames are
 * [U_mu | V_mu], its inner transfer tensors block-diagonal with blocks B_t at
 * (0,0,0) and F_t at (1,1,1), zero elsewhere, and its root the block-diagonal
 * matrix of alpha 2^(sA-s) B_D and beta 2^(sC-s) F_D with s = max(sA, sC).
 * A and C must share d and n.  S must have ranks rank_A + rank_C at every
 * non-root node, S->log2_scale is ignored on input and s is written to
 * *out_log2_scale (host).  Pure data movement: no floating-point arithmetic
 * except the two root scalings.  Errors: HT_EINVAL, HT_ESHAPE. */
ht_status ht_add(ht_context* ctx, double alpha, const ht_desc* A, double beta, const ht_desc* C,
                 const ht_desc* S, int64_t* out_log2_scale, void* stream);

/* ---------------------------------------------------------------- orthogonalisation
 * In-place bottom-up orthogonalisation of X (Section 3.4): leaves U <- Q of
 * the reduced QR U = QR (CholeskyQR2), inner nodes B <- (I,R_s1,R_s2) o B then
 * B <- Q^T of the QR of M_{2,3}(B) (eq. (qrtransfer)), root B_D <- R_t1 B_D R_t2^T.
 * Requires n_mu >= k_mu.  Each R is divided by a power of two; the new scale
 * exponent is written to out_log2_scale (DEVICE int64, required).  flags:
 * DEVICE uint32 or NULL.  Workspace: ht_orthogonalize_workspace() bytes,
 * 256-byte aligned.  Errors: HT_EINVAL, HT_ESHAPE, HT_EWORKSPACE, HT_EUNSUPPORTED. */
ht_status ht_orthogonalize_workspace(ht_context* ctx, const ht_desc* X, int32_t precision, size_t* bytes);
ht_status ht_orthogonalize(ht_context* ctx, const ht_desc* X, int32_t precision,
                           int64_t* out_log2_scale, uint32_t* flags,
                           void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- Gramians
 * Reduced Gramians Bhat_t = V_t^T V_t of an ORTHOGONAL tensor X (Section 3.3,
 * eqs. (acctransferroot), (acctransferSon1), (acctransferSon2)), top-down.
 * bhat[t] (DEVICE float64, k_t x k_t row-major) for every non-root t;
 * bhat[0] is ignored.  The Gramians are returned divided by 4^g with
 * g = e_D + log2_scale, e_D the binary exponent of ||B_D||_F (so their
 * traces are about 1); g is written to *out_log2_units (DEVICE int64, may be
 * NULL).  If sigma is not NULL, sigma[t] (DEVICE float64, k_t) receives the
 * square roots of the eigenvalues of Bhat_t in descending order, in the same
 * units (true singular value = sigma * 2^g).  Errors: as ht_orthogonalize. */
ht_status ht_gramians_workspace(ht_context* ctx, const ht_desc* X, size_t* bytes);
ht_status ht_gramians(ht_context* ctx, const ht_desc* X, double* const* bhat, double* const* sigma,
                      int64_t* out_log2_units, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- truncation (hot path)
 * Truncates the lazy sum S = sum_c coef[c] X[c] (n_in >= 1 summands with
 * equal d and n; n_in = 1 truncates one tensor) by the hierarchical SVD of
 * Section 3.3: orthogonalise S bottom-up (Section 3.4, CholeskyQR2 at the
 * leaves), form all reduced Gramians top-down, eigen-decompose them, choose
 * the ranks, and project: leaves U <- U Q|, inner nodes eq.
 * (transfertransformationtrunc), root B_D <- Q_t1|^T B_D Q_t2|.  The sum is
 * never materialised.
 * out: caller-allocated result with out->rank[t] equal to
 *   HT_RANK_FIXED: min(opts->ranks[t], K_t);
 *   HT_RANK_TOL:   min(K_t, max_rank) (an upper bound; the chosen r_t are
 *                  written to out_ranks and the output is zero beyond them,
 *                  so it represents the truncated tensor at either size).
 * out_ranks: DEVICE int32[2d-1] or NULL.  out_log2_scale: DEVICE int64,
 * required (the scale of the result).  flags: DEVICE uint32 or NULL.
 * out_sigma: DEVICE float64 [2d-1][128] or NULL: sigma_{t,i} / ||S|| in
 * descending order (row 0 unused).
 * Errors: HT_EINVAL, HT_ESHAPE, HT_EWORKSPACE, HT_EUNSUPPORTED. */
ht_status ht_truncate_workspace(ht_context* ctx, const ht_desc* X, int32_t n_in,
                                const ht_trunc_opts* opts, size_t* bytes);
ht_status ht_truncate(ht_context* ctx, const ht_desc* X, const double* coef, int32_t n_in,
                      const ht_trunc_opts* opts, const ht_desc* out, int32_t* out_ranks,
                      int64_t* out_log2_scale, uint32_t* flags, double* out_sigma,
                      void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- truncation without allocation
 * For callers that cannot allocate device memory: code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The same operation,
 * arguments, results and errors as ht_truncate, without the workspace: the
 * workspace and the launch tables live in a static device array of
 * HT_NOALLOC_SCRATCH_BYTES per GPU (the first 2 MiB hold the tables), which
 * every GPU the library runs on holds until the process ends.
 * ht_create_context() looks up the array's address on its device once.
 * The call allocates nothing (no hipMalloc or hipFree, no stream or event is
 * created; the whole tree runs on `stream`, and profiling takes no events
 * here).  Its launch tables are copied from host memory with hipMemcpyAsync
 * on `stream` unless the array already holds the same tables from the
 * previous call on this GPU.  The array keeps the last call's contents; every
 * call clears what it needs zeroed itself.  All calls on one GPU share the
 * array: calls that may overlap on the device (other streams or contexts
 * without ordering between them) race; calls on one stream are ordered.
 * Errors: as ht_truncate; HT_EWORKSPACE when the truncation needs more than
 * HT_NOALLOC_SCRATCH_BYTES - 2 MiB of workspace (ht_truncate_workspace gives
 * the figure) or more than 2 MiB of tables; HT_EUNSUPPORTED for device ids
 * above 63. */
#define HT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ht_status ht_truncate_noalloc(ht_context* ctx, const ht_desc* X, const double* coef, int32_t n_in,
                              const ht_trunc_opts* opts, const ht_desc* out, int32_t* out_ranks,
                              int64_t* out_log2_scale, uint32_t* flags, double* out_sigma, void* stream);

/* ---------------------------------------------------------------- batched truncation
 * Truncates `count` independent lazy sums in one pass: problem c is the sum of
 * X[o_c .. o_c + n_in[c]) (o_c = n_in[0] + .. + n_in[c-1]) with coefficients
 * coef[o_c ..] (coef may be NULL: all 1), options opts[c] and result out[c],
 * each exactly as for ht_truncate (Section 3.3, the same algorithm and the
 * same precision policy per problem).  Problems may differ in d, n, ranks,
 * dtypes, rank mode and precision.  The launches of the problems are merged
 * step by step (all leaf Grams of the batch in one launch, all Cholesky
 * factorisations of one level in one launch, ...), so the number of launches
 * does not grow with `count`.
 * out_ranks: host array [count] of DEVICE int32[2d_c-1] (the array or any
 * entry may be NULL).  out_log2_scale: DEVICE int64[count], required.  flags:
 * DEVICE uint32[count] or NULL.  out_sigma: host array [count] of DEVICE
 * float64 [2d_c-1][128] (the array or any entry may be NULL).  The results of
 * different problems must not overlap.  Workspace: the sum over the problems
 * of their ht_truncate_workspace() sizes, each rounded up to 256 bytes.
 * Errors: as ht_truncate; the message names the problem. */
ht_status ht_truncate_batched_workspace(ht_context* ctx, int32_t count, const ht_desc* X,
                                        const int32_t* n_in, const ht_trunc_opts* opts, size_t* bytes);
ht_status ht_truncate_batched(ht_context* ctx, int32_t count, const ht_desc* X, const int32_t* n_in,
                              const double* coef, const ht_trunc_opts* opts, const ht_desc* out,
                              int32_t* const* out_ranks, int64_t* out_log2_scale, uint32_t* flags,
                              double* const* out_sigma, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- inner product and norm
 * Inner product <X, Y> of two HT tensors on one tree (Section 3.2):
 * Definition (phi) bottom-up, Phi_mu = U_mu^T V_mu at the leaves, eq. (defphi)
 * Phi_t = M_1(B_t) (Phi_s1 (x) Phi_s2) M_1(F_t)^T at inner nodes (B of X, F
 * of Y) and <X, Y> = Phi_D at the root (Lemma (phi)).  X and Y must share d
 * and n; ranks and dtypes may differ.  The result is *out_val * 2^(*out_log2)
 * with 0.5 <= |*out_val| < 1, or 0 (out_val: DEVICE double, out_log2: DEVICE
 * int64, both required): every Phi_t is divided by a power of two on the way
 * up, so no range is exceeded.  Computed in float64.  flags: DEVICE uint32 or
 * NULL (bit 1: a non-finite value).  Workspace: ht_inner_workspace() bytes,
 * 256-byte aligned.  Errors: HT_EINVAL, HT_ESHAPE, HT_EWORKSPACE,
 * HT_EUNSUPPORTED (ranks above 128). */
ht_status ht_inner_workspace(ht_context* ctx, const ht_desc* X, const ht_desc* Y, size_t* bytes);
ht_status ht_inner(ht_context* ctx, const ht_desc* X, const ht_desc* Y, double* out_val, int64_t* out_log2,
                   uint32_t* flags, void* ws, size_t ws_bytes, void* stream);

/* Norm of the lazy sum S = sum_c coef[c] X[c] (n_in in [1, 8] summands with
 * equal d and n, coef NULL: all 1): S is orthogonalised bottom-up (Section
 * 3.4, the R factors only, float64) and ||S|| is the Frobenius norm of the
 * orthogonal root matrix.  With X = {A, B} and coef = {1, -1} this is the
 * difference norm ||A - B||, which does not suffer the cancellation of
 * <A,A> - 2<A,B> + <B,B>.  Result *out_val * 2^(*out_log2) as for ht_inner.
 * flags: DEVICE uint32 or NULL, as for ht_truncate.  Workspace:
 * ht_norm_workspace() bytes, 256-byte aligned.  Errors: as ht_truncate. */
ht_status ht_norm_workspace(ht_context* ctx, const ht_desc* X, int32_t n_in, size_t* bytes);
ht_status ht_norm(ht_context* ctx, const ht_desc* X, const double* coef, int32_t n_in, double* out_val,
                  int64_t* out_log2, uint32_t* flags, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- operator application
 * C = L A for an H-operator L and an H-tensor A on the same tree (Section
 * 3.6, Lemma (operator)).  L is passed as an ht_desc whose mode mu has
 * n_mu^2 rows (square operators): column r of its leaf frame is the matrix
 * W_{mu,r} (n_mu x n_mu) stored row-major, entry (j, i) at row j * n_mu + i
 * (the index pair (j_mu, i_mu) of eq. (operatorastensor)); its transfer
 * tensors H_t and root are as for any HT tensor.  C (caller-allocated) must
 * have A's mode sizes and ranks k^L_t k^A_t; C gets the leaf frames
 * V_mu[:, r k_mu + l] = W_{mu,r} U_mu[:, l] and the transfer tensors
 * F_t = H_t (x) B_t with F_t[(p,i)][(q,j)][(r,l)] = H_t[p][q][r] B_t[i][j][l]
 * (operator index slowest; the root likewise).  C's scale is not written:
 * the represented tensor is 2^(L.log2_scale + A.log2_scale) times C's data.
 * Products in float64; C may be float32 or float64.  No workspace.  Errors:
 * HT_EINVAL, HT_ESHAPE. */
ht_status ht_apply(ht_context* ctx, const ht_desc* L, const ht_desc* A, const ht_desc* C, void* stream);

/* ---------------------------------------------------------------- entries
 * A[i_1..i_d] for m multi-indices (Section 3.1): leaves pick row i_mu, inner
 * nodes apply eq. (transfermult), the root the root formula; evaluated level
 * by level for all indices at once.  idx: DEVICE int32, m x d row-major,
 * 0-based, each i_mu < n_mu (not checked on the device: out-of-range indices
 * are the caller's error).  out: DEVICE float64[m], scaled by 2^log2_scale
 * (entries beyond the float64 range become +-Inf or 0).  Computed in
 * float64.  Errors: HT_EINVAL, HT_EWORKSPACE. */
ht_status ht_entries_workspace(ht_context* ctx, const ht_desc* X, int64_t m, size_t* bytes);
ht_status ht_entries(ht_context* ctx, const ht_desc* X, int64_t m, const int32_t* idx, double* out,
                     void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- profiling
 * When enabled, every launch the library makes is bracketed by two HIP events
 * on the caller's stream.  ht_profile_read() waits for the recorded events,
 * folds them into per-(step, kernel) totals and returns up to max_entries of
 * them (*n_out = number available).  flops and bytes are the algorithmic
 * floating-point operations and the compulsory bytes (each operand read once,
 * each result written once) of the launches, fixed when the launch is planned.
 * ht_profile_reset() clears the totals.  Errors: HT_EINVAL, HT_EDEVICE. */
typedef struct {
  char label[48];             /* step of the method, e.g. "gramian_son1" */
  char kernel[48];            /* kernel launched, e.g. "gemm_kernel<float,double,double>" */
  int64_t launches;
  double ms;                  /* summed event time of those launches */
  double flops;
  double bytes;
} ht_profile_entry;
ht_status ht_profile_enable(ht_context* ctx, int32_t on);
ht_status ht_profile_read(ht_context* ctx, int32_t max_entries, ht_profile_entry* out, int32_t* n_out);
ht_status ht_profile_reset(ht_context* ctx);

#ifdef __cplusplus
}
#endif
#endif /* HT_H */
