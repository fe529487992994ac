// C ABI of the HT hierarchical-SVD library: argument checks, workspace layout,
// launch tables and the order of the launches.  Every floating-point step runs
// in the kernels of gemm.hip, smallla.hip and entries.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <list>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/ht.h"
#include "ht_internal.h"

using namespace ht;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static ht_status fail(ht_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HT_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(HT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

// ------------------------------------------------------------------ tree, eq. (balanced)
namespace ht {
Tree::Tree(int d_) : d(d_) {
  nn = 2 * d - 1;
  parent.assign(nn, -1); son1.assign(nn, -1); son2.assign(nn, -1);
  lo.assign(nn, 0); hi.assign(nn, 0); depth.assign(nn, 0); height.assign(nn, 0);
  leaf_node.assign(d, -1);
  int next = 0;
  // preorder visit of {mu..nu} (1-based): sons {mu..floor((mu+nu-1)/2)}, rest
  struct Frame { int mu, nu, par, dep; };
  std::vector<Frame> stack{{1, d, -1, 0}};
  std::vector<int> order;
  while (!stack.empty()) {
    Frame f = stack.back();
    stack.pop_back();
    const int t = next++;
    lo[t] = f.mu - 1; hi[t] = f.nu - 1; parent[t] = f.par; depth[t] = f.dep;
    if (f.par >= 0) {
      if (son1[f.par] < 0) son1[f.par] = t; else son2[f.par] = t;
    }
    if (f.mu < f.nu) {
      const int split = (f.mu + f.nu - 1) / 2;
      stack.push_back({split + 1, f.nu, t, f.dep + 1});  // second son visited after the first
      stack.push_back({f.mu, split, t, f.dep + 1});
    } else {
      leaf_node[f.mu - 1] = t;
    }
  }
  for (int t = nn - 1; t >= 0; --t)
    if (son1[t] >= 0) height[t] = 1 + std::max(height[son1[t]], height[son2[t]]);
}
int Tree::max_depth() const { return *std::max_element(depth.begin(), depth.end()); }
}  // namespace ht

// ------------------------------------------------------------------ launch plans
namespace {

enum OpKind : int {
  OP_GEMM, OP_CHOL1, OP_CHOL2, OP_EIG, OP_RANK, OP_PROJPREP, OP_ROOTNORM, OP_FILL, OP_SETSTATE,
  OP_WRITESCALE, OP_COPY, OP_SIGMA, OP_EGATHER, OP_ENORM, OP_EFINISH, OP_PHI, OP_KRON,
  OP_FORK,   // the library's second stream waits for the caller's stream here
  OP_JOIN    // the caller's stream waits for everything on the second stream
};

struct Op {
  int kind = 0;
  GemmLaunch g{};            // OP_GEMM (descs = table offset until bound)
  size_t toff = 0;           // table offset of descriptors / records
  int count = 0;
  size_t toff2 = 0;          // OP_RANK: table offset of the per-tensor StateRecs
  int count2 = 0;
  void* p0 = nullptr;        // generic pointers
  void* p1 = nullptr;
  void* p2 = nullptr;
  size_t bytes = 0;
  long long scale0 = 0;
  int i0 = 0, i1 = 0, i2 = 0, i3 = 0, i4 = 0, i5 = 0;
  double f0 = 0.0;
  int64_t c[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // OP_COPY: c[0] = largest record; entries: row count
  const char* label = "";    // step of the method this launch belongs to
  double flops = 0.0;        // algorithmic flops of the launch
  double bytes_alg = 0.0;    // compulsory bytes moved by the launch
  int tblocks = 4096;        // OP_GEMM: target workgroups of a split reduction
  bool sym_out = false;      // OP_GEMM: every result is symmetric
  bool acc64_req = false;    // OP_GEMM: float64 accumulation across k-slabs was asked for
  int stream = 0;            // 0: the caller's stream; 1: the library's second stream
};

// Label given to the launches added next (one per step of the method).
static thread_local const char* g_label = "";
// Stream of the launches added next (0: the caller's, 1: the second stream).
static thread_local int g_stream = 0;
struct Label {
  const char* prev;
  explicit Label(const char* l) : prev(g_label) { g_label = l; }
  ~Label() { g_label = prev; }
};

// Name of the kernel an op launches (as rocprof lists it, abbreviated).
static std::string kernel_name(const Op& op);

struct Plan {
  std::vector<Op> ops;
  std::vector<unsigned char> table;
  std::vector<unsigned char> key;
  void* dtable = nullptr;
  size_t dbytes = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Appends POD records to the host table image; returns their offset.
template <typename T>
size_t put(Plan& P, const std::vector<T>& v) {
  const size_t off = align256(P.table.size());
  P.table.resize(off + v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(P.table.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

int esize(int t) { return t == F32 ? 4 : 8; }

// algorithmic flops of one eigensolve with vectors, per K^3 (see add_small)
constexpr double kEigFlopsPerK3 = 4.0 / 3.0 + 4.0 / 3.0 + 2.0;


GemmDesc blank_desc() {
  GemmDesc d;
  std::memset(&d, 0, sizeof(d));
  d.KB = 1;
  d.nbatch = 1;
  d.alpha = 1.0;
  return d;
}

// Per-descriptor eligibility for the streamed kernel (small operand in LDS,
// the other streamed): -1 none, 0 with S = A, 1 with S = B^T.
int sb_want(const GemmDesc& d) {
  int kt = 0;
  if (d.nseg > 0) for (int s = 0; s < d.nseg; ++s) kt += d.segK[s];
  else kt = d.K;
  if (d.kr || d.KB != 1 || kt < 1 || kt > 128) return -1;
  const long long nbt = d.nbatch;
  // the streamed operand contiguous along its free index first; one
  // contiguous along the reduction also streams faster than the tiled kernels
  // take it (each lane's eight loads of a chunk cover 32 consecutive k)
  if (d.M <= 128 && d.sBn == 1 && d.N * nbt >= 256) return 0;   // S = A, T = B
  if (d.N <= 128 && d.sAm == 1 && d.M * nbt >= 256) return 1;   // S = B^T, T = A^T
  if (d.M <= 128 && d.N * nbt >= 256) return 0;
  if (d.N <= 128 && d.M * nbt >= 256) return 1;
  return -1;
}

// Shapes the split-K kernel takes (result at most 128 x 128, above 64 x 64).
bool rk_shape(const GemmDesc& d) {
  return !(d.kr || d.nseg > 0 || d.nbatch != 1 || d.M > 128 || d.N > 128 || d.M <= 64 || d.N <= 64 || d.K < 1 ||
           !(d.sAk == 1 || d.sAm == 1) || !(d.sBk == 1 || d.sBn == 1));
}

// B is A^T of the same matrix (a Gram matrix).
bool rk_gram(const GemmDesc& d) {
  return d.A == d.B && d.M == d.N && d.sAm == d.sBn && d.sAk == d.sBk && d.sAkb == d.sBkb;
}

// Adds one GEMM launch over `descs` (all sharing types, math, mode, layouts).
// The launch of a GEMM over `descs` (all sharing types, math, mode and
// layouts): kernel choice, tiling and split; the descriptors are not stored.
// sym_out: the caller knows that every result C is a symmetric matrix.
Op gemm_op(const std::vector<GemmDesc>& descs, int tA, int tB, int tC, int math, int mode, bool akc, bool bkc,
           bool acc64, int target_blocks, bool sym_out) {
  Op op;
  op.kind = OP_GEMM;
  op.tblocks = target_blocks;
  op.sym_out = sym_out;
  op.acc64_req = acc64;
  // large float64 problems use 128 x 128 tiles
  // (only when there are enough output tiles to fill the chip without
  // splitting the reduction; split-K problems keep 64 x 64 tiles)
  bool big = math == MATH_F64 && mode == GEMM_STORE;
  long long tiles128 = 0;
  for (const auto& d : descs) {
    if (d.kr || d.M < 96 || d.N < 96) big = false;
    tiles128 += (long long)((d.M + 127) / 128) * ((d.N + 127) / 128) * d.nbatch;
  }
  if (tiles128 < 512) big = false;
  // small x streamed: one operand at most 128 x 128 (whole reduction), the
  // other long and contiguous along its free index
  {
    bool ok = math == MATH_F64 && mode == GEMM_STORE;
    int swap = -1;
    long long items = 0;
    bool k64 = true, four = true;
    for (const auto& d : descs) {
      if (!ok) break;
      int kt = 0;
      if (d.nseg > 0) for (int s = 0; s < d.nseg; ++s) kt += d.segK[s];
      else kt = d.K;
      if (kt % 64) k64 = false;
      if (kt <= 96) four = false;   // four 32-deep chunks: the ring kernel
      const int want = sb_want(d);
      if (want < 0 || (swap >= 0 && want != swap)) { ok = false; break; }
      swap = want;
      const int ns = swap ? d.M : d.N;
      items = std::max<long long>(items, (long long)((ns + 127) / 128) * d.nbatch);
    }
    if (ok) {
      op.g.sb = true;
      big = false;
      op.g.sb_swap = swap == 1;
      op.g.sb_wn = 1;
      op.g.sb_cd = k64 ? 64 : 32;
      op.g.sb_ring = four;
      int rows = 0;   // largest row count of the small operand
      for (const auto& d : descs) rows = std::max(rows, op.g.sb_swap ? d.N : d.M);
      op.g.sb_rows = rows;
      const long long per = (512 + (long long)descs.size() - 1) / (long long)descs.size();
      op.g.sb_grid = (int)std::max<long long>(1, std::min(per, items));
    }
  }
  // long reductions into a result of at most 128 x 128, split over k
  // (only float64 results that are symmetric: a Gram matrix, where B is A^T,
  // or a result the caller declares symmetric; for the others the 64 x 64
  // tiles are as fast)
  if (mode == GEMM_ATOMIC && !op.g.sb && math == MATH_F64) {
    bool ok = true, sym = tA == tB;
    long long chunks = 0;
    for (const auto& d : descs) {
      if (!rk_shape(d)) { ok = false; break; }
      if (!rk_gram(d)) sym = false;
      chunks = std::max<long long>(chunks, (long long)((d.K + 15) / 16) * d.KB);
    }
    if (ok && (sym || sym_out)) {
      for (const auto& d : descs)
        if (d.M != d.N) ok = false;
    }
    if (ok && (sym || sym_out)) {
      op.g.rk = true;
      op.g.rk_sym = sym ? 1 : 2;
      op.g.rk_part = false;
      for (const auto& d : descs) op.g.rk_part = op.g.rk_part || std::max(d.M, d.N) <= 112;
      op.g.rk_kc = sym ? 32 : 16;
      // split-K width: about 512 workgroups, one round at two per CU
      const long long want = (512 + (long long)descs.size() - 1) / (long long)descs.size();
      op.g.rk_split = (int)std::max<long long>(1, std::min(want, (chunks + 15) / 16));
      big = false;
    }
  }
  const int tile = big ? 128 : 64;
  int maxtiles = 0, maxbatch = 1, maxkt = 1;
  for (const auto& d : descs) {
    const int tiles = ((d.M + tile - 1) / tile) * ((d.N + tile - 1) / tile);
    maxtiles = std::max(maxtiles, tiles);
    maxbatch = std::max(maxbatch, d.nbatch);
    int kt = 0;
    if (d.nseg > 0) for (int s = 0; s < d.nseg; ++s) kt += (d.segK[s] + 15) / 16;
    else kt = d.KB * ((d.K + 15) / 16);
    maxkt = std::max(maxkt, kt);
  }
  int split = 1;
  if (mode == GEMM_ATOMIC) {
    const long long base = (long long)maxtiles * maxbatch * (long long)descs.size();
    split = (int)std::max<long long>(1, std::min<long long>((target_blocks + base - 1) / base, maxkt / 4));
    split = std::max(1, std::min(split, 256));
  }
  op.g.tA = tA; op.g.tB = tB; op.g.tC = tC; op.g.math = math; op.g.mode = mode;
  op.g.a_kcontig = akc; op.g.b_kcontig = bkc;
  op.g.acc64 = acc64 && math == MATH_F32;
  op.g.big = big;
  op.g.splitk = split;
  op.g.ndesc = (int)descs.size();
  op.g.maxbatch = maxbatch;
  op.g.maxtiles = maxtiles;
  op.label = g_label;
  for (const auto& d : descs) {
    double kt = 0.0;
    if (d.nseg > 0) for (int s = 0; s < d.nseg; ++s) kt += d.segK[s];
    else kt = (double)d.KB * d.K;
    const double nb = d.nbatch;
    op.flops += 2.0 * nb * d.M * d.N * kt;
    op.bytes_alg += nb * ((double)d.M * kt * (tA == F32 ? 4 : 8) + kt * d.N * (tB == F32 ? 4 : 8) +
                          (double)d.M * d.N * (tC == F32 ? 4 : 8));
  }
  op.count = (int)descs.size();
  return op;
}

void add_gemm(Plan& P, const std::vector<GemmDesc>& descs, int tA, int tB, int tC, int math, int mode,
              bool akc, bool bkc, bool acc64 = false, int target_blocks = 4096, bool sym_out = false) {
  if (descs.empty()) return;
  Op op = gemm_op(descs, tA, tB, tC, math, mode, akc, bkc, acc64, target_blocks, sym_out);
  op.toff = put(P, descs);
  op.stream = g_stream;
  P.ops.push_back(op);
}

void add_small(Plan& P, int kind, const std::vector<SmallArgs>& a) {
  if (a.empty()) return;
  Op op;
  op.kind = kind;
  op.label = g_label;
  for (const auto& x : a) {
    op.i0 = std::max(op.i0, (int)x.K);   // the largest order (OP_EIG picks its kernel by it)
    op.bytes_alg += 2.0 * 8.0 * x.K * x.K;
    const double k3 = (double)x.K * x.K * x.K;
    // operation counts: symmetric eigensolver with vectors (Householder
    // tridiagonalisation 4/3 K^3, the divide-and-conquer eigenvector products
    // about 4/3 K^3, back-transformation 2 K^3); Cholesky K^3/3 and triangular
    // inverse K^3/3, and in the second step the two triangular products,
    // K^3/3 each
    if (kind == OP_EIG) op.flops += kEigFlopsPerK3 * k3;
    if (kind == OP_CHOL1 || kind == OP_CHOL2) op.flops += 2.0 / 3.0 * k3;
    if (kind == OP_CHOL2) op.flops += 2.0 / 3.0 * k3;
  }
  op.toff = put(P, a);
  op.count = (int)a.size();
  op.stream = g_stream;
  P.ops.push_back(op);
}

void add_fills(Plan& P, const std::vector<FillRec>& r) {
  size_t mx = 0;
  for (const auto& f : r) mx = std::max(mx, f.bytes);
  if (!mx) return;
  Op op; op.kind = OP_FILL; op.toff = put(P, r); op.count = (int)r.size(); op.bytes = mx; op.label = g_label;
  op.stream = g_stream;
  for (const auto& f : r) op.bytes_alg += (double)f.bytes;
  P.ops.push_back(op);
}

void add_fill(Plan& P, void* ptr, size_t bytes) {
  if (!bytes) return;
  add_fills(P, {FillRec{ptr, bytes}});
}

void add_copies(Plan& P, const std::vector<CopyRec>& r) {
  int64_t mx = 0;
  for (const auto& c : r) mx = std::max<int64_t>(mx, c.n0 * c.n1 * c.n2);
  if (mx <= 0) return;
  Op op; op.kind = OP_COPY; op.toff = put(P, r); op.count = (int)r.size(); op.c[0] = mx; op.label = g_label;
  op.stream = g_stream;
  for (const auto& c : r) op.bytes_alg += (double)(c.n0 * c.n1 * c.n2) * (esize(c.tsrc) + esize(c.tdst));
  P.ops.push_back(op);
}

void add_copy3(Plan& P, const void* src, int tsrc, void* dst, int tdst, int64_t n0, int64_t n1, int64_t n2,
               int64_t s0, int64_t s1, int64_t s2, int64_t d0, int64_t d1, int64_t d2, double alpha) {
  CopyRec c;
  std::memset(&c, 0, sizeof(c));
  c.src = src; c.dst = dst; c.tsrc = tsrc; c.tdst = tdst;
  c.n0 = n0; c.n1 = n1; c.n2 = n2; c.s0 = s0; c.s1 = s1; c.s2 = s2; c.d0 = d0; c.d1 = d1; c.d2 = d2;
  c.alpha = alpha;
  add_copies(P, {c});
}

void add_copy(Plan& P, const void* src, int tsrc, void* dst, int tdst, int64_t rows, int64_t cols,
              int64_t srs, int64_t scs, int64_t drs, int64_t dcs, double alpha) {
  add_copy3(P, src, tsrc, dst, tdst, 1, rows, cols, 0, srs, scs, 0, drs, dcs, alpha);
}

StateRec blank_state(GlobalState* st) {
  StateRec r;
  std::memset(&r, 0, sizeof(r));
  r.st = st;
  return r;
}

// One state op (OP_SETSTATE, OP_ROOTNORM, OP_WRITESCALE) over per-tensor records.
void add_state(Plan& P, int kind, const std::vector<StateRec>& r) {
  if (r.empty()) return;
  Op op; op.kind = kind; op.toff = put(P, r); op.count = (int)r.size(); op.label = g_label;
  op.stream = g_stream;
  P.ops.push_back(op);
}

// Fork to or join from the second stream.
void add_phi(Plan& P, const std::vector<PhiRec>& r) {
  if (r.empty()) return;
  Op op;
  op.kind = OP_PHI;
  op.count = (int)r.size();
  op.toff = put(P, r);
  op.label = g_label;
  op.stream = g_stream;
  P.ops.push_back(op);
}

void add_kron(Plan& P, const std::vector<KronRec>& r) {
  if (r.empty()) return;
  Op op;
  op.kind = OP_KRON;
  op.count = (int)r.size();
  for (const auto& k : r) {
    const double nF = (double)k.P * k.Q * k.R * k.I * k.J * k.L;
    op.c[0] = std::max<int64_t>(op.c[0], (int64_t)nF);
    op.c[1] = std::max<int64_t>(op.c[1], (int64_t)k.P * k.I);   // mode-1 index pairs (p, i)
    // one product per element of F; compulsory traffic: H and B read once, F written once
    op.flops += nF;
    op.bytes_alg += (double)k.P * k.Q * k.R * esize(k.tH) + (double)k.I * k.J * k.L * esize(k.tB) +
                    nF * esize(k.tF);
  }
  op.toff = put(P, r);
  op.label = g_label;
  op.stream = g_stream;
  P.ops.push_back(op);
}

PhiRec blank_phi() {
  PhiRec r;
  std::memset(&r, 0, sizeof(r));
  return r;
}

void add_sync(Plan& P, int kind) {
  Op op; op.kind = kind; op.label = kind == OP_FORK ? "fork" : "join";
  P.ops.push_back(op);
}

// The launches of one GEMM step over many problems (a batch of tensors): the
// descriptors are grouped by the kernel that suits each one alone (small
// operand in LDS with the other streamed, split-K symmetric, tiled), and each
// group is cut so that its grid stays within the launch limits (the tiled
// kernels put descriptors x batch on the third grid axis).
void add_gemm_grouped(Plan& P, const std::vector<GemmDesc>& descs, const Op& proto) {
  const GemmLaunch& q = proto.g;
  auto decide = [&](const std::vector<GemmDesc>& v) {
    return gemm_op(v, q.tA, q.tB, q.tC, q.math, q.mode, q.a_kcontig, q.b_kcontig, proto.acc64_req,
                   proto.tblocks, proto.sym_out);
  };
  // the kernel gemm_op would pick for the descriptor alone; streamed
  // products also by ring eligibility (reduction above 96) and, below it, by
  // the row blocks of the small operand, so that a launch of small problems
  // does not take the row count of the largest
  constexpr int kTiled = 1000;
  std::map<int, std::vector<GemmDesc>> cls;
  for (const auto& d : descs) {
    int c = kTiled;
    if (q.math == MATH_F64 && q.mode == GEMM_STORE) {
      const int w = sb_want(d);
      if (w >= 0) {
        int kt = 0;
        if (d.nseg > 0) for (int sg = 0; sg < d.nseg; ++sg) kt += d.segK[sg];
        else kt = d.K;
        const int rows = w ? d.N : d.M;
        c = 10 + 10 * w + (kt > 96 ? 0 : 1 + (rows + 31) / 32);
      }
    } else if (q.math == MATH_F64 && q.mode == GEMM_ATOMIC && rk_shape(d) && d.M == d.N) {
      const bool gram = q.tA == q.tB && rk_gram(d);
      if (gram || proto.sym_out) c = gram ? 2 : 3;
    }
    cls[c].push_back(d);
  }
  constexpr long long kGridMax = 65535;
  // 128-column items of a streamed product
  auto sb_items = [](const GemmDesc& d) {
    const int w = sb_want(d);
    const long long ns = w == 1 ? d.M : d.N;
    return (ns + 127) / 128 * (long long)d.nbatch;
  };
  for (auto& kv : cls) {
    auto& v = kv.second;
    const bool tiled = kv.first == kTiled;   // only the tiled kernels put the batch on a grid axis
    const bool streamed = kv.first >= 10 && kv.first < kTiled;
    // streamed products of many problems: the largest first (workgroups start
    // in index order), so that the launch does not end on one big product
    if (streamed)
      std::stable_sort(v.begin(), v.end(),
                       [&](const GemmDesc& a, const GemmDesc& b) { return sb_items(a) > sb_items(b); });
    // split-K Grams the same way, by reduction work
    const bool splitk = kv.first == 2 || kv.first == 3;
    auto rk_work = [](const GemmDesc& d) { return (double)d.M * d.N * d.K * d.KB; };
    if (splitk)
      std::stable_sort(v.begin(), v.end(),
                       [&](const GemmDesc& a, const GemmDesc& b) { return rk_work(a) > rk_work(b); });
    size_t i = 0;
    while (i < v.size()) {
      std::vector<GemmDesc> chunk;
      long long mb = 1;
      while (i < v.size()) {
        const long long nb = tiled ? std::max<long long>(mb, v[i].nbatch) : 1;
        if (!chunk.empty() && (long long)(chunk.size() + 1) * nb > kGridMax) break;
        mb = nb;
        chunk.push_back(v[i++]);
      }
      Op op = decide(chunk);
      if (op.g.sb) {
        // at least about 2048 workgroups over the launch: with one workgroup
        // per descriptor a product of 70 items would run on one CU while the
        // others idle; the surplus workgroups of small products exit at once
        long long most = 1;
        for (const auto& d : chunk) most = std::max(most, sb_items(d));
        const long long per = (2048 + (long long)chunk.size() - 1) / (long long)chunk.size();
        op.g.sb_grid = (int)std::max<long long>(op.g.sb_grid, std::min(per, most));
      }
      if (op.g.rk) {
        // likewise for the split-K Grams: at least about 2048 workgroups, each
        // still at least 16 chunks of 16 deep (a one-workgroup reduction over
        // 9216 terms had run on one CU)
        long long chunks = 1;
        for (const auto& d : chunk) chunks = std::max<long long>(chunks, (long long)((d.K + 15) / 16) * d.KB);
        const long long per = (2048 + (long long)chunk.size() - 1) / (long long)chunk.size();
        op.g.rk_split = (int)std::max<long long>(op.g.rk_split, std::min(per, (chunks + 15) / 16));
      }
      op.label = proto.label;
      op.stream = proto.stream;
      op.toff = put(P, chunk);
      P.ops.push_back(op);
    }
  }
}

// Interleaves the launch plans of independent problems (the tensors of a
// batch) into one plan whose launches each serve every problem at the same
// step.  A step is identified by (kind, label, stream, occurrence of that
// triple in its plan).  The plans are consumed from their heads: at each turn the step taken
// is one that no plan still holds behind its head, so the launches of one step
// are merged whole; each plan's own order is kept, which is all its
// correctness needs (the problems share no written memory).
// Node arguments of a merged one-workgroup-per-node launch (Cholesky,
// eigensolver) ordered by decreasing order K: workgroups start in index
// order, so the costliest nodes (cost ~ K^3) start first and the launch ends
// on small ones (longest-processing-time-first).  The nodes of such a launch
// are independent, so the order changes no result.
static void sort_largest_first(std::vector<SmallArgs>& v) {
  std::stable_sort(v.begin(), v.end(), [](const SmallArgs& a, const SmallArgs& b) { return a.K > b.K; });
}

ht_status merge_plans(const std::vector<Plan>& plans, Plan& M) {
  const int n = (int)plans.size();
  // steps as integer ids: (kind, label, stream, occurrence in the plan)
  std::map<std::string, int> ids;
  std::vector<std::vector<int>> key(n);
  for (int p = 0; p < n; ++p) {
    std::map<std::string, int> occ;
    for (const Op& op : plans[p].ops) {
      const std::string base =
          std::to_string(op.kind) + "|" + (op.label ? op.label : "") + "|" + std::to_string(op.stream);
      const std::string k = base + "|" + std::to_string(occ[base]++);
      auto it = ids.emplace(k, (int)ids.size()).first;
      key[p].push_back(it->second);
    }
  }
  // a step may be taken when every plan that still holds it holds it at its
  // head: left[k] (plans not yet past k) equals at_head[k]
  const int nk = (int)ids.size();
  std::vector<int> left(nk, 0), at_head(nk, 0), head(n, 0);
  for (int p = 0; p < n; ++p)
    for (int k : key[p]) ++left[k];
  auto done = [&](int p) { return head[p] >= (int)key[p].size(); };
  for (int p = 0; p < n; ++p)
    if (!done(p)) ++at_head[key[p][0]];
  while (true) {
    int first = -1;
    for (int p = 0; p < n && first < 0; ++p)
      if (!done(p)) first = p;
    if (first < 0) break;
    int chosen = -1;
    for (int p = first; p < n && chosen < 0; ++p)
      if (!done(p) && left[key[p][head[p]]] == at_head[key[p][head[p]]]) chosen = key[p][head[p]];
    if (chosen < 0) chosen = key[first][head[first]];
    std::vector<std::pair<int, const Op*>> grp;
    for (int p = 0; p < n; ++p)
      if (!done(p) && key[p][head[p]] == chosen) {
        grp.push_back({p, &plans[p].ops[head[p]]});
        --left[chosen];
        --at_head[chosen];
        ++head[p];
        if (!done(p)) ++at_head[key[p][head[p]]];
      }
    const Op& o0 = *grp[0].second;
    auto tab = [&](int p, size_t off) { return plans[p].table.data() + off; };
    switch (o0.kind) {
      case OP_GEMM: {
        // one merged step per set of launch parameters
        std::vector<bool> used(grp.size(), false);
        for (size_t i = 0; i < grp.size(); ++i) {
          if (used[i]) continue;
          const Op& a = *grp[i].second;
          std::vector<GemmDesc> ds;
          for (size_t j = i; j < grp.size(); ++j) {
            const Op& b = *grp[j].second;
            if (used[j] || b.g.tA != a.g.tA || b.g.tB != a.g.tB || b.g.tC != a.g.tC || b.g.math != a.g.math ||
                b.g.mode != a.g.mode || b.g.a_kcontig != a.g.a_kcontig || b.g.b_kcontig != a.g.b_kcontig ||
                b.acc64_req != a.acc64_req || b.tblocks != a.tblocks || b.sym_out != a.sym_out)
              continue;
            used[j] = true;
            const GemmDesc* src = reinterpret_cast<const GemmDesc*>(tab(grp[j].first, b.toff));
            ds.insert(ds.end(), src, src + b.count);
          }
          add_gemm_grouped(M, ds, a);
        }
        break;
      }
      case OP_CHOL1: case OP_CHOL2: case OP_EIG: case OP_PROJPREP: case OP_RANK: {
        std::vector<SmallArgs> sa;
        std::vector<StateRec> sr;
        Op op = o0;
        op.flops = op.bytes_alg = 0.0;
        for (const auto& pr : grp) {
          const Op& b = *pr.second;
          const SmallArgs* src = reinterpret_cast<const SmallArgs*>(tab(pr.first, b.toff));
          const int a0 = (int)sa.size();
          for (int j = 0; j < b.count; ++j) {
            SmallArgs a = src[j];
            if (!a.st) a.st = reinterpret_cast<GlobalState*>(b.p0);
            if (!a.st) return fail(HT_EUNSUPPORTED, "batched plan: node arguments without their tensor state");
            sa.push_back(a);
          }
          if (b.kind == OP_RANK) {
            const StateRec* rs = reinterpret_cast<const StateRec*>(tab(pr.first, b.toff2));
            for (int j = 0; j < b.count2; ++j) {
              StateRec r = rs[j];
              r.a0 += a0;
              sr.push_back(r);
            }
          }
          op.flops += b.flops;
          op.bytes_alg += b.bytes_alg;
        }
        if (o0.kind == OP_EIG) {
          // the eigensolver by order: nodes up to 96 run two to a CU
          std::vector<SmallArgs> lo, mid, hi;
          for (const auto& x : sa) (x.K <= 64 ? lo : (x.K <= 96 ? mid : hi)).push_back(x);
          for (auto* part : {&lo, &mid, &hi}) {
            if (part->empty()) continue;
            sort_largest_first(*part);
            Op e = op;
            e.toff = put(M, *part);
            e.count = (int)part->size();
            e.i0 = 0;
            e.flops = e.bytes_alg = 0.0;
            for (const auto& x : *part) {
              e.i0 = std::max(e.i0, (int)x.K);
              e.bytes_alg += 2.0 * 8.0 * x.K * x.K;
              e.flops += kEigFlopsPerK3 * (double)x.K * x.K * x.K;
            }
            M.ops.push_back(e);
          }
          break;
        }
        if (o0.kind == OP_CHOL1 || o0.kind == OP_CHOL2) sort_largest_first(sa);
        op.toff = put(M, sa);
        op.count = (int)sa.size();
        if (o0.kind == OP_RANK) {
          op.toff2 = put(M, sr);
          op.count2 = (int)sr.size();
        }
        M.ops.push_back(op);
        break;
      }
      case OP_FORK: case OP_JOIN:
        add_sync(M, o0.kind);
        break;
      case OP_FILL: {
        std::vector<FillRec> r;
        for (const auto& pr : grp) {
          const FillRec* src = reinterpret_cast<const FillRec*>(tab(pr.first, pr.second->toff));
          r.insert(r.end(), src, src + pr.second->count);
        }
        const char* l = g_label;
        const int sm = g_stream;
        g_label = o0.label;
        g_stream = o0.stream;
        add_fills(M, r);
        g_label = l;
        g_stream = sm;
        break;
      }
      case OP_COPY: {
        std::vector<CopyRec> r;
        for (const auto& pr : grp) {
          const CopyRec* src = reinterpret_cast<const CopyRec*>(tab(pr.first, pr.second->toff));
          r.insert(r.end(), src, src + pr.second->count);
        }
        const char* l = g_label;
        const int sm = g_stream;
        g_label = o0.label;
        g_stream = o0.stream;
        add_copies(M, r);
        g_label = l;
        g_stream = sm;
        break;
      }
      case OP_SETSTATE: case OP_ROOTNORM: case OP_WRITESCALE: {
        std::vector<StateRec> r;
        for (const auto& pr : grp) {
          const StateRec* src = reinterpret_cast<const StateRec*>(tab(pr.first, pr.second->toff));
          r.insert(r.end(), src, src + pr.second->count);
        }
        const char* l = g_label;
        const int sm = g_stream;
        g_label = o0.label;
        g_stream = o0.stream;
        add_state(M, o0.kind, r);
        g_label = l;
        g_stream = sm;
        break;
      }
      default:
        return fail(HT_EUNSUPPORTED, "batched plan: launch kind " + std::to_string(o0.kind) + " cannot be merged");
    }
  }
  return HT_OK;
}

// The cache key of a plan: every field of every launch, appended one by one
// (the structs themselves hold padding whose bytes are not defined), then
// the argument table (its records are cleared before they are filled, so
// their padding is zero).
template <typename T>
static void key_put(std::vector<unsigned char>& k, const T& v) {
  const unsigned char* b = reinterpret_cast<const unsigned char*>(&v);
  k.insert(k.end(), b, b + sizeof(T));
}

void build_key(Plan& P) {
  std::vector<unsigned char>& k = P.key;
  k.clear();
  k.reserve(P.ops.size() * 256 + P.table.size());
  for (const Op& op : P.ops) {
    key_put(k, op.kind);
    const GemmLaunch& g = op.g;
    const int gi[] = {g.tA, g.tB, g.tC, g.math, g.mode, (int)g.a_kcontig, (int)g.b_kcontig, g.splitk,
                      (int)g.acc64, (int)g.big, (int)g.sb, (int)g.sb_swap, g.sb_grid, g.sb_wn, g.sb_cd,
                      (int)g.sb_ring, g.sb_rows, (int)g.rk_part, (int)g.rk, g.rk_sym, g.rk_split, g.rk_kc,
                      g.ndesc, g.maxbatch, g.maxtiles};
    for (int x : gi) key_put(k, x);
    key_put(k, op.toff); key_put(k, op.count); key_put(k, op.toff2); key_put(k, op.count2);
    key_put(k, op.p0); key_put(k, op.p1); key_put(k, op.p2);
    key_put(k, op.bytes); key_put(k, op.scale0);
    const int oi[] = {op.i0, op.i1, op.i2, op.i3, op.i4, op.i5, op.tblocks, (int)op.sym_out,
                      (int)op.acc64_req, op.stream};
    for (int x : oi) key_put(k, x);
    key_put(k, op.f0);
    for (int64_t c : op.c) key_put(k, c);
    key_put(k, op.label);
  }
  k.insert(k.end(), P.table.begin(), P.table.end());
}

}  // namespace

struct ProfPending { hipEvent_t a, b; const char* label; std::string kernel; double flops, bytes; };
struct ProfAgg { std::string label, kernel; long long n = 0; double ms = 0, flops = 0, bytes = 0; };

struct ht_context {
  int device = 0;
  std::mutex mu;
  std::mutex run_mu;                     // one plan at a time uses the second stream (taken after mu)
  hipStream_t side = nullptr;            // second stream (default priority), created on first use
  std::vector<hipEvent_t> sync_events;   // fork / join events
  // the last batched call: its argument signature, merged plan and table
  std::vector<unsigned char> bsig;
  Plan bplan;
  void* btable = nullptr;
  std::list<Plan> cache;   // most recent first
  bool prof = false;
  std::vector<hipEvent_t> free_events;
  std::vector<ProfPending> pending;
  std::vector<ProfAgg> agg;
};

static hipEvent_t take_event(ht_context* c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

namespace {

const size_t kCacheMax = 24;

ht_status launch_plan(ht_context* ctx, const Plan& P, void* dtable, hipStream_t stream, bool allow_prof = true);

ht_status run_plan(ht_context* ctx, Plan& P, hipStream_t stream) {
  build_key(P);
  void* dtable = nullptr;
  // the lock is held through the enqueue: a concurrent call could otherwise
  // evict and free this table before its launches are queued
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (auto it = ctx->cache.begin(); it != ctx->cache.end(); ++it) {
    if (it->key == P.key) {
      dtable = it->dtable;
      ctx->cache.splice(ctx->cache.begin(), ctx->cache, it);
      break;
    }
  }
  if (!dtable && !P.table.empty()) {
    if (ctx->cache.size() >= kCacheMax) {
      HT_HIP(hipDeviceSynchronize());
      (void)hipFree(ctx->cache.back().dtable);
      ctx->cache.pop_back();
    }
    HT_HIP(hipMalloc(&dtable, P.table.size()));
    const hipError_t e = hipMemcpy(dtable, P.table.data(), P.table.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(dtable);
      return fail(HT_EDEVICE, std::string("plan table upload: ") + hipGetErrorString(e));
    }
    Plan c;
    c.key = P.key;
    c.dtable = dtable;
    c.dbytes = P.table.size();
    ctx->cache.push_front(std::move(c));
  }
  return launch_plan(ctx, P, dtable, stream);
}

// Enqueues the launches of a plan whose argument table is at dtable.  With
// allow_prof false no timing events are taken, even when profiling is on.
ht_status launch_plan(ht_context* ctx, const Plan& P, void* dtable, hipStream_t stream, bool allow_prof) {
  char* tb = reinterpret_cast<char*>(dtable);
  const bool prof = ctx->prof && allow_prof;
  bool forks = false;
  for (const auto& op : P.ops) forks = forks || op.kind == OP_FORK;
  std::unique_lock<std::mutex> run_lk;
  if (forks) {
    run_lk = std::unique_lock<std::mutex>(ctx->run_mu);
    if (!ctx->side) HT_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
  }
  size_t nsync = 0;
  for (const auto& op : P.ops) {
    if (op.kind == OP_FORK || op.kind == OP_JOIN) {
      if (nsync == ctx->sync_events.size()) {
        hipEvent_t ev = nullptr;
        HT_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        ctx->sync_events.push_back(ev);
      }
      hipEvent_t ev = ctx->sync_events[nsync++];
      hipStream_t from = op.kind == OP_FORK ? stream : ctx->side, to = op.kind == OP_FORK ? ctx->side : stream;
      HT_HIP(hipEventRecord(ev, from));
      HT_HIP(hipStreamWaitEvent(to, ev, 0));
      continue;
    }
    const hipStream_t ostream = stream;
    if (op.stream) stream = ctx->side;
    hipError_t e = hipSuccess;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof) {
      ev0 = take_event(ctx);
      ev1 = take_event(ctx);
      if (ev0) (void)hipEventRecord(ev0, stream);
    }
    switch (op.kind) {
      case OP_GEMM: {
        GemmLaunch g = op.g;
        g.descs = reinterpret_cast<const GemmDesc*>(tb + op.toff);
        e = launch_gemm(g, stream);
        break;
      }
      case OP_CHOL1:
      case OP_CHOL2:
        e = launch_chol(reinterpret_cast<const SmallArgs*>(tb + op.toff), op.count,
                        op.kind == OP_CHOL1 ? 1 : 2, stream, reinterpret_cast<GlobalState*>(op.p0));
        break;
      case OP_EIG:
        e = launch_eig(reinterpret_cast<const SmallArgs*>(tb + op.toff), op.count, op.i0, stream,
                       reinterpret_cast<GlobalState*>(op.p0));
        break;
      case OP_RANK:
        e = launch_rank_select(reinterpret_cast<const SmallArgs*>(tb + op.toff),
                               reinterpret_cast<const StateRec*>(tb + op.toff2), op.count2, stream);
        break;
      case OP_PROJPREP:
        e = launch_proj_prep(reinterpret_cast<const SmallArgs*>(tb + op.toff), op.count,
                             reinterpret_cast<const GlobalState*>(op.p0), stream);
        break;
      case OP_SIGMA:
        e = launch_sigma_from_lam(reinterpret_cast<const SmallArgs*>(tb + op.toff), op.count,
                                  reinterpret_cast<double* const*>(tb + op.bytes), stream);
        break;
      case OP_ROOTNORM:
        e = launch_root_norm(reinterpret_cast<const StateRec*>(tb + op.toff), op.count, stream);
        break;
      case OP_FILL:
        e = launch_fill(reinterpret_cast<const FillRec*>(tb + op.toff), op.count, op.bytes, stream);
        break;
      case OP_SETSTATE:
        e = launch_set_state(reinterpret_cast<const StateRec*>(tb + op.toff), op.count, stream);
        break;
      case OP_WRITESCALE:
        e = launch_write_scale(reinterpret_cast<const StateRec*>(tb + op.toff), op.count, stream);
        break;
      case OP_EGATHER:
        e = launch_entry_gather(reinterpret_cast<const EntryNode*>(tb + op.toff), op.count, op.c[0],
                                reinterpret_cast<const int32_t*>(op.p0), op.i0, 0, stream);
        break;
      case OP_ENORM:
        e = launch_entry_normalize(reinterpret_cast<const EntryNode*>(tb + op.toff), op.count, op.c[0], 0, stream);
        break;
      case OP_EFINISH:
        e = launch_entry_finish(reinterpret_cast<const double*>(op.p0), reinterpret_cast<const int32_t*>(op.p1),
                                op.c[0], op.scale0, reinterpret_cast<double*>(op.p2), stream);
        break;
      case OP_COPY:
        e = launch_copy3(reinterpret_cast<const CopyRec*>(tb + op.toff), op.count, op.c[0], stream);
        break;
      case OP_PHI:
        e = launch_phi_scale(reinterpret_cast<const PhiRec*>(tb + op.toff), op.count, stream);
        break;
      case OP_KRON:
        e = launch_kron(reinterpret_cast<const KronRec*>(tb + op.toff), op.count, op.c[0], op.c[1], stream);
        break;
    }
    if (e != hipSuccess) return fail(HT_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    if (prof && ev0 && ev1) {
      (void)hipEventRecord(ev1, stream);
      const std::string kn = kernel_name(op);
      ctx->pending.push_back({ev0, ev1, (op.label && *op.label) ? op.label : "other", kn, op.flops, op.bytes_alg});
    }
    stream = ostream;
  }
  return HT_OK;
}

std::string kernel_name(const Op& op) {
  auto tn = [](int t) { return t == F32 ? "float" : "double"; };
  switch (op.kind) {
    case OP_GEMM:   // the template arguments of the kernel that launch_gemm picks
      if (op.g.sb && op.g.sb_ring) {
        const int ts = op.g.sb_swap ? op.g.tB : op.g.tA, tt = op.g.sb_swap ? op.g.tA : op.g.tB;
        return std::string("gemm_sb_ring_kernel<") + tn(ts) + "," + tn(tt) + "," + tn(op.g.tC) + ">";
      }
      if (op.g.sb) {
        const int ts = op.g.sb_swap ? op.g.tB : op.g.tA, tt = op.g.sb_swap ? op.g.tA : op.g.tB;
        const int nrb = op.g.sb_rows <= 32 ? 2 : op.g.sb_rows <= 64 ? 4 : op.g.sb_rows <= 96 ? 6 : 8;
        return std::string("gemm_sb_kernel<") + tn(ts) + "," + tn(tt) + ",1," + std::to_string(op.g.sb_cd == 64 ? 64 : 32) +
               "," + std::to_string(nrb) + ">";
      }
      if (op.g.rk) {
        const std::string tm = op.g.math == MATH_F32 ? "float" : "double";
        const int kc = op.g.rk_sym == 1 ? 32 : 16;
        const bool km = op.g.rk_sym == 2 && !op.g.a_kcontig && !op.g.b_kcontig;
        return std::string("gemm_rk_kernel<") + tn(op.g.tA) + "," + tn(op.g.tB) + "," + tm + "," +
               std::to_string(op.g.rk_sym) + "," + std::to_string(kc) + "," + (km ? "true" : "false") +
               (op.g.rk_part ? ",true" : ",false") + ">";
      }
      if (op.g.big) return std::string("gemm128_kernel<") + tn(op.g.tA) + "," + tn(op.g.tB) + ">";
      return std::string("gemm_kernel<") + tn(op.g.tA) + "," + tn(op.g.tB) + "," +
             (op.g.math == MATH_F32 ? "float" : "double") + "," +
             (op.g.math == MATH_F32 && op.g.acc64 ? "true" : "false") + ">";
    case OP_CHOL1: case OP_CHOL2: return "chol_kernel";
    case OP_EIG: return op.i0 <= 64 ? "eig_kernel<64>" : (op.i0 <= 96 ? "eig_kernel<96>" : "eig_kernel<128>");
    case OP_RANK: return "rank_kernel";
    case OP_PROJPREP: return "proj_prep_kernel";
    case OP_SIGMA: return "sigma_kernel";
    case OP_ROOTNORM: return "root_norm_kernel";
    case OP_FILL: return "fill_kernel";
    case OP_SETSTATE: return "set_state_kernel";
    case OP_WRITESCALE: return "write_scale_kernel";
    case OP_COPY: return "copy3_kernel";
    case OP_EGATHER: return "gather_kernel";
    case OP_ENORM: return "normalize_kernel";
    case OP_EFINISH: return "finish_kernel";
    case OP_PHI: return "phi_scale_kernel";
    case OP_KRON: return "kron_kernel";
    case OP_FORK: return "fork";
    case OP_JOIN: return "join";
  }
  return "?";
}

// ------------------------------------------------------------------ validation
ht_status check_desc(const ht_desc* X, const char* name, bool need_data = true) {
  if (!X) return fail(HT_EINVAL, std::string(name) + " is NULL");
  if (X->d < 2) return fail(HT_EINVAL, std::string(name) + ": d must be >= 2");
  if (X->d > 4096) return fail(HT_EUNSUPPORTED, std::string(name) + ": d > 4096");
  if (!X->n || !X->rank) return fail(HT_EINVAL, std::string(name) + ": n or rank is NULL");
  if (X->frame_dtype != HT_F32 && X->frame_dtype != HT_F64) return fail(HT_EINVAL, std::string(name) + ": bad frame_dtype");
  if (X->transfer_dtype != HT_F32 && X->transfer_dtype != HT_F64)
    return fail(HT_EINVAL, std::string(name) + ": bad transfer_dtype");
  if (need_data && (!X->leaf || !X->leaf_ld || !X->transfer))
    return fail(HT_EINVAL, std::string(name) + ": leaf, leaf_ld or transfer is NULL");
  Tree tr(X->d);
  for (int mu = 0; mu < X->d; ++mu) {
    if (X->n[mu] < 1) return fail(HT_EINVAL, std::string(name) + ": n_mu must be >= 1");
    if (X->n[mu] > (int64_t)1 << 31) return fail(HT_EUNSUPPORTED, std::string(name) + ": n_mu too large");
    if (need_data) {
      if (!X->leaf[mu]) return fail(HT_EINVAL, std::string(name) + ": leaf pointer is NULL");
      if (X->leaf_ld[mu] < X->n[mu]) return fail(HT_EINVAL, std::string(name) + ": leaf_ld < n_mu");
    }
  }
  for (int t = 1; t < tr.nn; ++t) {
    if (X->rank[t] < 1) return fail(HT_EINVAL, std::string(name) + ": ranks must be >= 1");
    if (need_data && !tr.is_leaf(t) && !X->transfer[t]) return fail(HT_EINVAL, std::string(name) + ": transfer pointer is NULL");
  }
  if (need_data && !X->transfer[0]) return fail(HT_EINVAL, std::string(name) + ": root pointer is NULL");
  return HT_OK;
}

// ------------------------------------------------------------------ bump allocator over a workspace
// Address ranges known to the bounds validator (debug builds of a plan only).
struct Region { uintptr_t lo; size_t bytes; std::string what; };
static thread_local std::vector<Region>* g_regions = nullptr;
static void reg(const void* p, size_t bytes, const std::string& what) {
  if (g_regions && p && bytes) g_regions->push_back({reinterpret_cast<uintptr_t>(p), bytes, what});
}

struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(void* b) : base(reinterpret_cast<char*>(b)) {}
  void* take(size_t bytes) {
    off = align256(off);
    void* p = base ? base + off : reinterpret_cast<void*>(off + 256);  // dry run: fake non-null
    off += bytes;
    if (base) reg(p, bytes, "workspace");
    return p;
  }
};

// Per-node buffers of the truncation / orthogonalisation.
struct NodeBufs {
  int K = 0, rcap = 0;
  double *G = nullptr, *G2 = nullptr, *Bh = nullptr, *R1 = nullptr, *Ri1 = nullptr, *R = nullptr,
         *Ri = nullptr, *Q = nullptr, *lam = nullptr, *Qm = nullptr, *scratch = nullptr;
  void *Rf = nullptr, *QmT = nullptr, *Pm = nullptr;
  int32_t* rank = nullptr;
  double* Y = nullptr;      // leaves: n x K sweep-2 temporary; inner: K x K1K2
  void* Bp = nullptr;       // inner: (I, R_s1, R_s2) o H_t
  void* Tmp = nullptr;      // inner: mode-3 intermediate
  void* Qo = nullptr;       // inner: orthogonal transfer tensor
  double* C = nullptr;      // inner: (Bhat_t, I, I) o Qo
  void* E1 = nullptr;
  void* E2 = nullptr;
};

struct SumInfo {
  int n_in = 1;
  std::vector<const ht_desc*> X;
  std::vector<double> alpha;      // root coefficients incl. scale differences
  long long scale0 = 0;
  std::vector<int> K;             // sum rank per node
  std::vector<std::vector<int>> off;  // off[t][c]: offset of summand c in the sum rank
};

ht_status sum_info(const ht_desc* X, const double* coef, int n_in, SumInfo& S) {
  if (n_in < 1 || n_in > MAX_SEG) return fail(HT_EINVAL, "n_in must be in [1, 8]");
  for (int c = 0; c < n_in; ++c) {
    ht_status st = check_desc(&X[c], "X[c]");
    if (st) return st;
    if (X[c].d != X[0].d) return fail(HT_ESHAPE, "summands must share d");
    for (int mu = 0; mu < X[0].d; ++mu)
      if (X[c].n[mu] != X[0].n[mu]) return fail(HT_ESHAPE, "summands must share n");
    if (X[c].frame_dtype != X[0].frame_dtype || X[c].transfer_dtype != X[0].transfer_dtype)
      return fail(HT_ESHAPE, "summands must share dtypes");
  }
  S.n_in = n_in;
  const int d = X[0].d, nn = 2 * d - 1;
  S.X.resize(n_in);
  long long smax = X[0].log2_scale;
  for (int c = 0; c < n_in; ++c) { S.X[c] = &X[c]; smax = std::max<long long>(smax, X[c].log2_scale); }
  S.scale0 = smax;
  S.alpha.resize(n_in);
  for (int c = 0; c < n_in; ++c) {
    const double cf = coef ? coef[c] : 1.0;
    if (!std::isfinite(cf)) return fail(HT_EINVAL, "coefficients must be finite");
    S.alpha[c] = std::ldexp(cf, (int)std::max<long long>(-2000, X[c].log2_scale - smax));
  }
  S.K.assign(nn, 0);
  S.off.assign(nn, std::vector<int>(n_in, 0));
  for (int t = 1; t < nn; ++t)
    for (int c = 0; c < n_in; ++c) {
      S.off[t][c] = S.K[t];
      S.K[t] += X[c].rank[t];
    }
  S.K[0] = 1;
  for (int t = 1; t < nn; ++t)
    if (S.K[t] > KMAX) return fail(HT_EUNSUPPORTED, "sum rank above 128 at node " + std::to_string(t));
  return HT_OK;
}

// Bottom-up orthogonalisation of the lazy sum (Section 3.4) into `B`.
// Leaves: CholeskyQR2 of W = [U^(1) | ... | U^(n_in)].  Inner nodes:
// Bp = (I, R_s1, R_s2) o H_t, CholeskyQR2 of M_{2,3}(Bp), Qo = R_t^{-T} M_1(Bp).
// Root: BDo = R_t1 H_D R_t2^T.
struct OrthOut {
  std::vector<NodeBufs> nb;
  double* HD = nullptr;
  double* BDo = nullptr;
  double* T1 = nullptr;
  GlobalState* st = nullptr;
};

// overlap: each level's orthogonal factor Qo (read only by the Gramian pass)
// is formed on the second stream while the next level's first Cholesky step
// (a few workgroups) leaves the chip idle; the caller's stream waits for it
// at the end.
// form_qo: false when only the R factors and the root are wanted (a norm).
void plan_orth(Plan& P, const Tree& tr, const SumInfo& S, int prec, Arena& A, OrthOut& O,
               const std::vector<int>& rcap, bool need_proj_bufs, const ht_desc* out,
               const ht_desc* inplace, bool overlap = false, bool form_qo = true) {
  const int nn = tr.nn, d = tr.d;
  // Precision policy.  The first CholeskyQR2 sweeps (leaf frames and M_{2,3}
  // of every transfer tensor) run on the FP32 matrix cores in the mixed path:
  // the float64 second sweep removes their error.  Every other product, and
  // all storage, is float64: at d = 64 each float32 stage of the forward
  // contractions or projections adds a few 1e-7 to the relative error of the
  // truncated tensor, and together they exceed 1e-6.
  const int T = F64;                                          // storage / forward-product type
  const int fmath = MATH_F64;                                 // forward products
  const int smath = prec == HT_PREC_MIXED ? MATH_F32 : MATH_F64;  // first sweeps
  const int tsz = esize(T);
  const ht_desc& X0 = *S.X[0];
  O.nb.assign(nn, NodeBufs());
  // ---- zero region (atomic accumulation targets)
  size_t z0 = align256(A.off);
  A.off = z0;
  for (int t = 1; t < nn; ++t) {
    NodeBufs& b = O.nb[t];
    b.K = S.K[t];
    const size_t kk = (size_t)b.K * b.K * 8;
    b.G = (double*)A.take(kk);
    b.G2 = (double*)A.take(kk);
    b.Bh = (double*)A.take(kk);
  }
  O.HD = (double*)A.take((size_t)S.K[tr.son1[0]] * S.K[tr.son2[0]] * 8);
  const size_t zbytes = A.off - z0;
  void* zptr = A.base ? A.base + z0 : nullptr;
  reg(zptr, zbytes, "zero region");
  O.st = (GlobalState*)A.take(sizeof(GlobalState));
  // ---- the rest
  for (int t = 1; t < nn; ++t) {
    NodeBufs& b = O.nb[t];
    const size_t kk = (size_t)b.K * b.K;
    b.rcap = rcap.empty() ? b.K : rcap[t];
    b.R1 = (double*)A.take(kk * 8);
    b.Ri1 = (double*)A.take(kk * 8);
    b.R = (double*)A.take(kk * 8);
    b.Ri = (double*)A.take(kk * 8);
    b.Rf = A.take(kk * tsz);
    if (need_proj_bufs) {
      b.Q = (double*)A.take(kk * 8);
      b.lam = (double*)A.take(b.K * 8);
      b.Qm = (double*)A.take((size_t)b.K * b.rcap * 8);
      b.QmT = A.take((size_t)b.K * b.rcap * tsz);
      b.rank = (int32_t*)A.take(4);
      b.scratch = (double*)A.take(eig_scratch_doubles(b.K) * 8);
    }
    if (tr.is_leaf(t)) {
      const int64_t n = X0.n[tr.mode(t)];
      b.Y = (double*)A.take((size_t)n * b.K * 8);
      if (need_proj_bufs) b.Pm = A.take((size_t)b.K * b.rcap * tsz);
    } else {
      const int K1 = S.K[tr.son1[t]], K2 = S.K[tr.son2[t]];
      const size_t vol = (size_t)b.K * K1 * K2;
      b.Bp = A.take(vol * tsz);
      size_t tmpn = 0;
      for (int c = 0; c < S.n_in; ++c)
        tmpn += (size_t)S.X[c]->rank[t] * S.X[c]->rank[tr.son1[t]] * K2;
      b.Tmp = A.take(tmpn * tsz);
      b.Y = (double*)A.take(vol * 8);
      if (form_qo) b.Qo = A.take(vol * tsz);
      if (need_proj_bufs) {
        b.C = (double*)A.take(vol * 8);
      }
    }
  }
  const int K1r = S.K[tr.son1[0]], K2r = S.K[tr.son2[0]];
  O.BDo = (double*)A.take((size_t)K1r * K2r * 8);
  O.T1 = (double*)A.take((size_t)K1r * K2r * 8);
  for (int t = 1; t < nn; ++t) {
    NodeBufs& b = O.nb[t];
    if (need_proj_bufs && !tr.is_leaf(t)) {
      const int K1 = S.K[tr.son1[t]], K2 = S.K[tr.son2[t]];
      b.E1 = A.take((size_t)b.rcap * K1 * K2 * tsz);
      b.E2 = A.take((size_t)b.rcap * rcap[tr.son1[t]] * K2 * tsz);
    }
  }

  // ---- launches
  g_label = "setup";
  {
    StateRec r = blank_state(O.st);
    r.scale0 = S.scale0;
    add_state(P, OP_SETSTATE, {r});
  }
  add_fill(P, zptr, zbytes);

  const int fdt = X0.frame_dtype, tdt = X0.transfer_dtype;
  g_label = "leaf_gram_sweep1";
  // leaves: sweep 1 Gram G = W^T W.  Two frames with one row stride form one
  // float64 Gram matrix of the split-K kernel (rows of the second frame at a
  // fixed element offset); otherwise the Gram matrix is formed in blocks of
  // summand pairs.
  {
    std::vector<GemmDesc> ds, dw;
    const int64_t es = esize(fdt);
    for (int mu = 0; mu < d; ++mu) {
      const int t = tr.leaf_node[mu];
      if (S.n_in == 2) {
        const int r0 = S.X[0]->rank[t], r1 = S.X[1]->rank[t];
        const int64_t ld = S.X[0]->leaf_ld[mu];
        const int64_t diff = (int64_t)((const char*)S.X[1]->leaf[mu] - (const char*)S.X[0]->leaf[mu]);
        GemmDesc g = blank_desc();
        g.A = S.X[0]->leaf[mu]; g.sAm = ld; g.sAk = 1;
        g.B = g.A; g.sBk = 1; g.sBn = ld;
        g.a2off = diff / es - (int64_t)r0 * ld; g.msplit = r0;
        g.C = O.nb[t].G; g.sCm = S.K[t]; g.sCn = 1;
        g.M = g.N = r0 + r1; g.K = (int)X0.n[mu];
        if (S.X[1]->leaf_ld[mu] == ld && diff % es == 0 && r0 > 0 && r1 > 0 && S.off[t][1] == r0 &&
            S.K[t] == r0 + r1 && rk_shape(g) && rk_gram(g)) {
          dw.push_back(g);
          continue;
        }
      }
      for (int c1 = 0; c1 < S.n_in; ++c1)
        for (int c2 = 0; c2 < S.n_in; ++c2) {
          GemmDesc g = blank_desc();
          g.A = S.X[c1]->leaf[mu]; g.sAm = S.X[c1]->leaf_ld[mu]; g.sAk = 1;
          g.B = S.X[c2]->leaf[mu]; g.sBk = 1; g.sBn = S.X[c2]->leaf_ld[mu];
          g.C = O.nb[t].G + (size_t)S.off[t][c1] * S.K[t] + S.off[t][c2];
          g.sCm = S.K[t]; g.sCn = 1;
          g.M = S.X[c1]->rank[t]; g.N = S.X[c2]->rank[t]; g.K = (int)X0.n[mu];
          ds.push_back(g);
        }
    }
    // float64 MFMA: as fast here as float32, and exact products
    add_gemm(P, dw, fdt, fdt, F64, MATH_F64, GEMM_ATOMIC, true, true);
    add_gemm(P, ds, fdt, fdt, F64, smath, GEMM_ATOMIC, true, true);
  }
  // first sweeps shift G by 10 u (K + sqrt(rows)) trace(G), u the unit
  // roundoff of the sweep's Gram products: above the rounding error of G and
  // of its factorisation, so W R1^{-1} stays bounded for any W
  const double shift_unit = prec == HT_PREC_MIXED ? 0x1p-24 : 0x1p-53;
  auto sweep1_shift = [&](int t) {
    const double rows = tr.son1[t] < 0 ? (double)X0.n[tr.mode(t)]
                                       : (double)S.K[tr.son1[t]] * (double)S.K[tr.son2[t]];
    return 10.0 * shift_unit * ((double)S.K[t] + std::sqrt(rows));
  };
  auto small_args = [&](const std::vector<int>& nodes, double tol, bool shift = false) {
    std::vector<SmallArgs> v;
    for (int t : nodes) {
      NodeBufs& b = O.nb[t];
      SmallArgs a;
      std::memset(&a, 0, sizeof(a));
      a.K = b.K; a.node = t; a.rcap = b.rcap;
      a.G = b.G; a.G2 = b.G2; a.R1 = b.R1; a.Ri1 = b.Ri1;
      a.R = b.R; a.Ri = b.Ri; a.Rf = b.Rf;
      a.rf_type = T; a.tol_rel = tol;
      a.shift_rel = shift ? sweep1_shift(t) : 0.0;
      a.Q = b.Q; a.lam = b.lam; a.Qm = b.Qm; a.QmT = b.QmT; a.rank_dev = b.rank; a.scratch = b.scratch;
      a.Bh = b.Bh;
      a.st = O.st;
      v.push_back(a);
    }
    return v;
  };
  std::vector<int> leaves;
  for (int mu = 0; mu < d; ++mu) leaves.push_back(tr.leaf_node[mu]);
  {
    Op op;
    g_label = "leaf_chol1";
    auto a = small_args(leaves, prec == HT_PREC_MIXED ? 1e-5 : 1e-12, true);
    add_small(P, OP_CHOL1, a);
    P.ops.back().p0 = O.st;
  }
  // sweep 2: Y = W R1^{-1} (float64), G2 = Y^T Y
  {
    std::vector<GemmDesc> ds;
    for (int mu = 0; mu < d; ++mu) {
      const int t = tr.leaf_node[mu];
      GemmDesc g = blank_desc();
      g.nseg = S.n_in;
      for (int c = 0; c < S.n_in; ++c) {
        g.segA[c] = S.X[c]->leaf[mu];
        g.segAk[c] = S.X[c]->leaf_ld[mu];
        g.segBoff[c] = (int64_t)S.off[t][c] * S.K[t];
        g.segK[c] = S.X[c]->rank[t];
      }
      g.A = S.X[0]->leaf[mu]; g.sAm = 1;
      g.B = O.nb[t].Ri1; g.sBk = S.K[t]; g.sBn = 1;
      g.C = O.nb[t].Y; g.sCm = 1; g.sCn = X0.n[mu];
      g.M = (int)X0.n[mu]; g.N = S.K[t]; g.K = 0;
      ds.push_back(g);
    }
    g_label = "leaf_sweep2_form";
    add_gemm(P, ds, fdt, F64, F64, MATH_F64, GEMM_STORE, false, false);
    ds.clear();
    for (int mu = 0; mu < d; ++mu) {
      const int t = tr.leaf_node[mu];
      GemmDesc g = blank_desc();
      g.A = O.nb[t].Y; g.sAm = X0.n[mu]; g.sAk = 1;
      g.B = O.nb[t].Y; g.sBk = 1; g.sBn = X0.n[mu];
      g.C = O.nb[t].G2; g.sCm = S.K[t]; g.sCn = 1;
      g.M = S.K[t]; g.N = S.K[t]; g.K = (int)X0.n[mu];
      ds.push_back(g);
    }
    g_label = "leaf_sweep2_gram";
    add_gemm(P, ds, F64, F64, F64, MATH_F64, GEMM_ATOMIC, true, true);
  }
  {
    g_label = "leaf_chol2";
    auto a = small_args(leaves, 1e-13);
    add_small(P, OP_CHOL2, a);   // also R = R2 R1, Ri = R1^{-1} R2^{-1}, Rf
    P.ops.back().p0 = O.st;
  }
  // inner nodes by height
  bool forked = false;
  std::vector<GemmDesc> pending_dq;
  const int H = tr.height[0];
  for (int h = 1; h < H; ++h) {
    std::vector<int> nodes;
    for (int t = 1; t < nn; ++t)
      if (!tr.is_leaf(t) && tr.height[t] == h) nodes.push_back(t);
    if (nodes.empty()) continue;
    // mode-3: Tmp_c = B^(c) x_3 R_s2[:, o2 : o2+k2c]
    std::vector<GemmDesc> d3, d2;
    for (int t : nodes) {
      const int s1 = tr.son1[t], s2 = tr.son2[t];
      const int K1 = S.K[s1], K2 = S.K[s2];
      size_t toff = 0;
      for (int c = 0; c < S.n_in; ++c) {
        const int kt = S.X[c]->rank[t], k1 = S.X[c]->rank[s1], k2 = S.X[c]->rank[s2];
        GemmDesc g = blank_desc();
        g.A = S.X[c]->transfer[t]; g.sAm = k2; g.sAk = 1;
        g.B = (const char*)O.nb[s2].Rf + (size_t)S.off[s2][c] * tsz; g.sBk = 1; g.sBn = K2;
        void* tmpc = (char*)O.nb[t].Tmp + toff * tsz;
        g.C = tmpc; g.sCm = K2; g.sCn = 1;
        g.M = kt * k1; g.N = K2; g.K = k2;
        d3.push_back(g);
        // mode-2: Bp[o_t + i] = R_s1[:, o1 : o1+k1c] Tmp_c[i]
        GemmDesc h2 = blank_desc();
        h2.A = (const char*)O.nb[s1].Rf + (size_t)S.off[s1][c] * tsz; h2.sAm = K1; h2.sAk = 1;
        h2.B = tmpc; h2.sBk = K2; h2.sBn = 1; h2.sBb = (int64_t)k1 * K2;
        h2.C = (char*)O.nb[t].Bp + (size_t)S.off[t][c] * K1 * K2 * tsz; h2.sCm = K2; h2.sCn = 1;
        h2.sCb = (int64_t)K1 * K2;
        h2.M = K1; h2.N = K2; h2.K = k1; h2.nbatch = kt;
        d2.push_back(h2);
        toff += (size_t)kt * k1 * K2;
      }
    }
    g_label = "inner_mode3_R";
    add_gemm(P, d3, tdt, T, T, fmath, GEMM_STORE, true, true, true);
    g_label = "inner_mode2_R";
    add_gemm(P, d2, T, T, T, fmath, GEMM_STORE, true, false, true);
    // sweep 1: G = M1(Bp) M1(Bp)^T in float64
    std::vector<GemmDesc> dg;
    for (int t : nodes) {
      const int K1 = S.K[tr.son1[t]], K2 = S.K[tr.son2[t]];
      const int64_t w = (int64_t)K1 * K2;
      GemmDesc g = blank_desc();
      g.A = O.nb[t].Bp; g.sAm = w; g.sAk = 1;
      g.B = O.nb[t].Bp; g.sBk = 1; g.sBn = w;
      g.C = O.nb[t].G; g.sCm = S.K[t]; g.sCn = 1;
      g.M = S.K[t]; g.N = S.K[t]; g.K = (int)w;
      dg.push_back(g);
    }
    g_label = "inner_gram_sweep1";
    // the operands are float64 here; where the split-K Gram kernel takes the
    // shape, its FP64 matrix cores are faster than the FP32 kernels on these
    // shapes, so the mixed path uses them too
    bool rk_all = !dg.empty();
    for (const auto& g : dg) rk_all = rk_all && rk_shape(g) && rk_gram(g);
    add_gemm(P, dg, T, T, F64, rk_all ? MATH_F64 : smath, GEMM_ATOMIC, true, true);
    if (!pending_dq.empty()) {   // the previous level's Qo beside this level's Cholesky
      g_label = "inner_orth_factor";
      add_sync(P, OP_FORK);
      g_stream = 1;
      add_gemm(P, pending_dq, F64, T, T, MATH_F64, GEMM_STORE, false, false);
      g_stream = 0;
      pending_dq.clear();
      forked = true;
    }
    {
      g_label = "inner_chol1";
      auto a = small_args(nodes, prec == HT_PREC_MIXED ? 1e-5 : 1e-12, true);
      add_small(P, OP_CHOL1, a);
      P.ops.back().p0 = O.st;
    }
    // sweep 2: Y = R1^{-T} M1(Bp) (float64), G2 = Y Y^T
    std::vector<GemmDesc> dy, dg2, dq;
    for (int t : nodes) {
      const int K1 = S.K[tr.son1[t]], K2 = S.K[tr.son2[t]];
      const int64_t w = (int64_t)K1 * K2;
      GemmDesc g = blank_desc();
      g.A = O.nb[t].Ri1; g.sAm = 1; g.sAk = S.K[t];
      g.B = O.nb[t].Bp; g.sBk = w; g.sBn = 1;
      g.C = O.nb[t].Y; g.sCm = w; g.sCn = 1;
      g.M = S.K[t]; g.N = (int)w; g.K = S.K[t];
      dy.push_back(g);
      GemmDesc h = blank_desc();
      h.A = O.nb[t].Y; h.sAm = w; h.sAk = 1;
      h.B = O.nb[t].Y; h.sBk = 1; h.sBn = w;
      h.C = O.nb[t].G2; h.sCm = S.K[t]; h.sCn = 1;
      h.M = S.K[t]; h.N = S.K[t]; h.K = (int)w;
      dg2.push_back(h);
      GemmDesc q = blank_desc();
      q.A = O.nb[t].Ri; q.sAm = 1; q.sAk = S.K[t];
      q.B = O.nb[t].Bp; q.sBk = w; q.sBn = 1;
      const bool write_user = inplace != nullptr;
      q.C = write_user ? inplace->transfer[t] : O.nb[t].Qo; q.sCm = w; q.sCn = 1;
      q.M = S.K[t]; q.N = (int)w; q.K = S.K[t];
      dq.push_back(q);
    }
    g_label = "inner_sweep2_form";
    add_gemm(P, dy, F64, T, F64, MATH_F64, GEMM_STORE, false, false);
    g_label = "inner_sweep2_gram";
    add_gemm(P, dg2, F64, F64, F64, MATH_F64, GEMM_ATOMIC, true, true);
    {
      g_label = "inner_chol2";
      auto a = small_args(nodes, 1e-13);
      add_small(P, OP_CHOL2, a);   // also R = R2 R1, Ri = R1^{-1} R2^{-1}, Rf
      P.ops.back().p0 = O.st;
    }
    g_label = "inner_orth_factor";
    if (!form_qo)
      ;
    else if (overlap)
      pending_dq = dq;   // formed during the next level
    else
      add_gemm(P, dq, F64, T, inplace ? inplace->transfer_dtype : T, MATH_F64, GEMM_STORE, false, false);
  }
  if (!pending_dq.empty()) {   // the top level's Qo
    g_label = "inner_orth_factor";
    add_gemm(P, pending_dq, F64, T, T, MATH_F64, GEMM_STORE, false, false);
  }
  g_label = "root_orth";
  // root: HD = blockdiag(alpha_c B_D^(c)); BDo = R_t1 HD R_t2^T
  const int t1 = tr.son1[0], t2 = tr.son2[0];
  {
    std::vector<CopyRec> cr;
    for (int c = 0; c < S.n_in; ++c) {
      const int r1 = S.X[c]->rank[t1], r2 = S.X[c]->rank[t2];
      CopyRec q;
      std::memset(&q, 0, sizeof(q));
      q.src = S.X[c]->transfer[0]; q.tsrc = F64;
      q.dst = O.HD + (size_t)S.off[t1][c] * K2r + S.off[t2][c]; q.tdst = F64;
      q.n0 = 1; q.n1 = r1; q.n2 = r2; q.s1 = r2; q.s2 = 1; q.d1 = K2r; q.d2 = 1;
      q.alpha = S.alpha[c];
      cr.push_back(q);
    }
    add_copies(P, cr);
  }
  {
    std::vector<GemmDesc> a1, a2;
    GemmDesc g = blank_desc();
    g.A = O.nb[t1].R; g.sAm = K1r; g.sAk = 1;
    g.B = O.HD; g.sBk = K2r; g.sBn = 1;
    g.C = O.T1; g.sCm = K2r; g.sCn = 1;
    g.M = K1r; g.N = K2r; g.K = K1r;
    a1.push_back(g);
    add_gemm(P, a1, F64, F64, F64, MATH_F64, GEMM_STORE, true, false);
    GemmDesc h = blank_desc();
    h.A = O.T1; h.sAm = K2r; h.sAk = 1;
    h.B = O.nb[t2].R; h.sBk = 1; h.sBn = K2r;
    h.C = inplace ? inplace->transfer[0] : O.BDo; h.sCm = K2r; h.sCn = 1;
    h.M = K1r; h.N = K2r; h.K = K2r;
    a2.push_back(h);
    add_gemm(P, a2, F64, F64, F64, MATH_F64, GEMM_STORE, true, true);
  }
  if (forked) add_sync(P, OP_JOIN);
  (void)out;
}

// Top-down Gramians (eqs. (acctransferroot), (acctransferSon1/2)) from the
// orthogonal root BDo and orthogonal transfer tensors Qo[t] (type tq).
// after(dep), if given, is called once the Gramians of all nodes down to
// depth dep + 1 are planned.
void plan_gramians(Plan& P, const Tree& tr, const std::vector<int>& K, std::vector<NodeBufs>& nb,
                   const double* BDo, GlobalState* st, const std::vector<const void*>& Qo, int tq,
                   const std::function<void(int)>& after = nullptr) {
  const int t1 = tr.son1[0], t2 = tr.son2[0];
  const int K1r = K[t1], K2r = K[t2];
  g_label = "gramian_root";
  {
    StateRec r = blank_state(st);
    r.BD = BDo; r.K1 = K1r; r.K2 = K2r;
    add_state(P, OP_ROOTNORM, {r});
  }
  {
    std::vector<GemmDesc> a, b;
    GemmDesc g = blank_desc();
    g.A = BDo; g.sAm = K2r; g.sAk = 1;
    g.B = BDo; g.sBk = 1; g.sBn = K2r;
    g.C = nb[t1].Bh; g.sCm = K1r; g.sCn = 1;
    g.M = K1r; g.N = K1r; g.K = K2r; g.alpha_dev = &st->alpha_gram;
    a.push_back(g);
    add_gemm(P, a, F64, F64, F64, MATH_F64, GEMM_STORE, true, true);
    GemmDesc h = blank_desc();
    h.A = BDo; h.sAm = 1; h.sAk = K2r;
    h.B = BDo; h.sBk = K2r; h.sBn = 1;
    h.C = nb[t2].Bh; h.sCm = K2r; h.sCn = 1;
    h.M = K2r; h.N = K2r; h.K = K1r; h.alpha_dev = &st->alpha_gram;
    b.push_back(h);
    add_gemm(P, b, F64, F64, F64, MATH_F64, GEMM_STORE, false, false);
  }
  if (after) after(0);
  const int D = tr.max_depth();
  for (int dep = 1; dep < D; ++dep) {
    std::vector<GemmDesc> dc, ds1, ds2;
    for (int t = 1; t < tr.nn; ++t) {
      if (tr.is_leaf(t) || tr.depth[t] != dep) continue;
      const int s1 = tr.son1[t], s2 = tr.son2[t];
      const int Kt = K[t], K1 = K[s1], K2 = K[s2];
      const int64_t w = (int64_t)K1 * K2;
      GemmDesc g = blank_desc();
      g.A = nb[t].Bh; g.sAm = Kt; g.sAk = 1;
      g.B = Qo[t]; g.sBk = w; g.sBn = 1;
      g.C = nb[t].C; g.sCm = w; g.sCn = 1;
      g.M = Kt; g.N = (int)w; g.K = Kt;
      dc.push_back(g);
      // Bhat_s1[p,q] = sum_{i,l} Qo[i,p,l] C[i,q,l]
      GemmDesc h = blank_desc();
      h.A = Qo[t]; h.sAm = K2; h.sAk = 1; h.sAkb = w;
      h.B = nb[t].C; h.sBk = 1; h.sBn = K2; h.sBkb = w;
      h.C = nb[s1].Bh; h.sCm = K1; h.sCn = 1;
      h.M = K1; h.N = K1; h.K = K2; h.KB = Kt;
      ds1.push_back(h);
      // Bhat_s2[p,q] = sum_{i,j} Qo[i,j,p] C[i,j,q]
      GemmDesc q = blank_desc();
      q.A = Qo[t]; q.sAm = 1; q.sAk = K2;
      q.B = nb[t].C; q.sBk = K2; q.sBn = 1;
      q.C = nb[s2].Bh; q.sCm = K2; q.sCn = 1;
      q.M = K2; q.N = K2; q.K = Kt * K1;
      ds2.push_back(q);
    }
    g_label = "gramian_mode1";
    add_gemm(P, dc, F64, tq, F64, MATH_F64, GEMM_STORE, true, false);
    // the son Gramians are symmetric because Bhat_t is
    g_label = "gramian_son1";
    add_gemm(P, ds1, tq, F64, F64, MATH_F64, GEMM_ATOMIC, true, true, false, 4096, true);
    g_label = "gramian_son2";
    add_gemm(P, ds2, tq, F64, F64, MATH_F64, GEMM_ATOMIC, false, false, false, 4096, true);
    if (after) after(dep);
  }
}

}  // namespace

// ------------------------------------------------------------------ static scratch
// Workspace and launch tables of ht_truncate_noalloc: one array per GPU,
// loaded with the library's code object and held until the process ends.
// In host code `scratch` names a host-side stand-in; kernels only ever get
// the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[HT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr size_t kNoAllocTableBytes = size_t(2) << 20;   // launch tables at the front
constexpr int kNoAllocDevices = 64;
struct NoAllocDevice {
  std::mutex mu;                        // one enqueue at a time on this GPU
  void* ptr = nullptr;                  // device address of `scratch` on this GPU
  std::vector<unsigned char> table;     // the table image last copied to the array
};
NoAllocDevice g_noalloc[kNoAllocDevices];

// Looks up this device's copy of the array (device must be current).
ht_status noalloc_setup(int device) {
  if (device < 0 || device >= kNoAllocDevices) return HT_OK;   // the entry point reports it
  NoAllocDevice& nd = g_noalloc[device];
  std::lock_guard<std::mutex> lk(nd.mu);
  if (nd.ptr) return HT_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(HT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  nd.ptr = p;
  return HT_OK;
}
}  // namespace

// ================================================================== ABI
extern "C" {

int32_t ht_version(void) { return 1; }

const char* ht_status_string(ht_status s) {
  switch (s) {
    case HT_OK: return "ok";
    case HT_EINVAL: return "invalid argument";
    case HT_ESHAPE: return "inconsistent shapes";
    case HT_EWORKSPACE: return "workspace too small or misaligned";
    case HT_EDEVICE: return "HIP runtime error";
    case HT_EUNSUPPORTED: return "unsupported size";
  }
  return "unknown status";
}

const char* ht_last_error(void) { return g_last_error.c_str(); }

ht_status ht_create_context(int device, ht_context** out) {
  if (!out) return fail(HT_EINVAL, "out is NULL");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return fail(HT_EDEVICE, "no such HIP device");
  int prev = 0;
  HT_HIP(hipGetDevice(&prev));
  HT_HIP(hipSetDevice(device));
  const ht_status st = noalloc_setup(device);
  (void)hipSetDevice(prev);
  if (st) return st;
  ht_context* c = new ht_context();
  c->device = device;
  *out = c;
  return HT_OK;
}

void ht_destroy_context(ht_context* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  for (auto& p : ctx->cache) (void)hipFree(p.dtable);
  for (auto& p : ctx->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto& e : ctx->free_events) (void)hipEventDestroy(e);
  for (auto& e : ctx->sync_events) (void)hipEventDestroy(e);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->btable) (void)hipFree(ctx->btable);
  delete ctx;
}

ht_status ht_tree(int32_t d, int32_t* parent, int32_t* son1, int32_t* son2, int32_t* lo, int32_t* hi,
                  int32_t* depth, int32_t* height) {
  if (d < 2) return fail(HT_EINVAL, "d must be >= 2");
  Tree tr(d);
  for (int t = 0; t < tr.nn; ++t) {
    if (parent) parent[t] = tr.parent[t];
    if (son1) son1[t] = tr.son1[t];
    if (son2) son2[t] = tr.son2[t];
    if (lo) lo[t] = tr.lo[t];
    if (hi) hi[t] = tr.hi[t];
    if (depth) depth[t] = tr.depth[t];
    if (height) height[t] = tr.height[t];
  }
  return HT_OK;
}

// ------------------------------------------------------------------ truncation
// overlap: run the upper part of the tree on the library's second stream
// (see below); off for the plans of a batch, which are merged instead.
// used (optional): the workspace bytes the plan takes (as need reports).
static ht_status build_truncate(ht_context* ctx, const ht_desc* X, const double* coef, int32_t n_in,
                                const ht_trunc_opts* opts, const ht_desc* out, int32_t* out_ranks,
                                int64_t* out_scale, uint32_t* flags, double* out_sigma, void* ws,
                                Plan& P, size_t* need, bool overlap = true, size_t* used = nullptr) {
  (void)ctx;
  if (!opts) return fail(HT_EINVAL, "opts is NULL");
  if (opts->mode != HT_RANK_FIXED && opts->mode != HT_RANK_TOL) return fail(HT_EINVAL, "bad rank mode");
  if (opts->precision != HT_PREC_FP64 && opts->precision != HT_PREC_MIXED) return fail(HT_EINVAL, "bad precision");
  if (opts->mode == HT_RANK_FIXED && !opts->ranks) return fail(HT_EINVAL, "opts->ranks is NULL");
  if (opts->mode == HT_RANK_TOL && !(opts->eps >= 0.0)) return fail(HT_EINVAL, "eps must be >= 0");
  if (!X) return fail(HT_EINVAL, "X is NULL");
  SumInfo S;
  ht_status st = sum_info(X, coef, n_in, S);
  if (st) return st;
  const int d = X[0].d;
  Tree tr(d);
  const int nn = tr.nn;
  std::vector<int> rcap(nn, 1);
  for (int t = 1; t < nn; ++t) {
    if (opts->mode == HT_RANK_FIXED) {
      if (opts->ranks[t] < 1) return fail(HT_EINVAL, "fixed ranks must be >= 1");
      rcap[t] = std::min(opts->ranks[t], S.K[t]);
    } else {
      rcap[t] = opts->max_rank > 0 ? std::min(opts->max_rank, S.K[t]) : S.K[t];
    }
  }
  if (opts->mode == HT_RANK_TOL) {  // the sons of the root share one rank
    const int r = std::min(rcap[tr.son1[0]], rcap[tr.son2[0]]);
    rcap[tr.son1[0]] = rcap[tr.son2[0]] = r;
  }
  if (!need) {
    st = check_desc(out, "out");
    if (st) return st;
    if (out->d != d) return fail(HT_ESHAPE, "out->d differs");
    for (int mu = 0; mu < d; ++mu)
      if (out->n[mu] != X[0].n[mu]) return fail(HT_ESHAPE, "out->n differs");
    for (int t = 1; t < nn; ++t)
      if (out->rank[t] != rcap[t])
        return fail(HT_ESHAPE, "out->rank[" + std::to_string(t) + "] must be " + std::to_string(rcap[t]));
    if (!out_scale) return fail(HT_EINVAL, "out_log2_scale is NULL");
  }
  const int prec = opts->precision;
  const int T = F64;            // storage and forward products: see plan_orth
  const int fmath = MATH_F64;
  const int tsz = esize(T);
  Arena A(ws);
  OrthOut O;
  plan_orth(P, tr, S, prec, A, O, rcap, true, out, nullptr, overlap);
  std::vector<const void*> Qo(nn, nullptr);
  for (int t = 1; t < nn; ++t) Qo[t] = O.nb[t].Qo;
  // Node groups.  An eigensolver launch lasts as long as one node's
  // decomposition, whatever the number of nodes.  With overlap, the upper
  // group (every non-root node above the deepest level) is decomposed on the
  // second stream as soon as its Gramians exist, and the projections that
  // need upper eigenvectors only (the root, inner nodes with upper sons,
  // upper leaves) follow it there, while the caller's stream forms the last
  // Gramian level and decomposes the lower group.  The rank rule of the
  // lower group reuses the threshold the upper group computed (the sons of
  // the root, which give ||A||, are upper).
  const int Dmax = tr.max_depth();
  const bool split = overlap && Dmax >= 2;
  std::vector<char> upper(nn, 0);
  std::vector<int> up_nodes, low_nodes;
  for (int t = 1; t < nn; ++t) {
    upper[t] = split && tr.depth[t] <= Dmax - 1;
    (upper[t] ? up_nodes : low_nodes).push_back(t);
  }
  auto node_args = [&](const std::vector<int>& nodes) {
    std::vector<SmallArgs> sa;
    for (int t : nodes) {
      NodeBufs& b = O.nb[t];
      SmallArgs a;
      std::memset(&a, 0, sizeof(a));
      a.K = b.K; a.node = t; a.rcap = b.rcap; a.rfix = opts->mode == HT_RANK_FIXED ? rcap[t] : 0;
      a.Q = b.Q; a.lam = b.lam; a.Qm = b.Qm; a.QmT = b.QmT; a.rf_type = T;
      a.rank_dev = out_ranks ? out_ranks + t : b.rank;
      a.scratch = b.scratch; a.Bh = b.Bh;
      a.sigma_out = out_sigma ? out_sigma + (size_t)t * KMAX : nullptr;
      a.st = O.st;
      sa.push_back(a);
    }
    return sa;
  };
  auto emit_eig = [&](const std::vector<int>& nodes, const char* label) {
    if (nodes.empty()) return;
    g_label = label;
    add_small(P, OP_EIG, node_args(nodes));
    P.ops.back().p0 = O.st;
  };
  auto emit_rank_prep = [&](const std::vector<int>& nodes, const char* l_rank, const char* l_prep) {
    if (nodes.empty()) return;
    const std::vector<SmallArgs> sa = node_args(nodes);
    g_label = l_rank;
    add_small(P, OP_RANK, sa);
    {
      StateRec r = blank_state(O.st);
      r.a0 = 0; r.na = (int)sa.size(); r.d = d; r.mode = opts->mode; r.eps = opts->eps;
      r.rel = opts->eps_relative ? 1 : 0; r.t1 = tr.son1[0]; r.t2 = tr.son2[0];
      Op& op = P.ops.back();
      op.toff2 = put(P, std::vector<StateRec>{r});
      op.count2 = 1;
    }
    g_label = l_prep;
    add_small(P, OP_PROJPREP, sa);
    P.ops.back().p0 = O.st;
  };
  // projections (eq. (nodewisetruncation), eq. (transfertransformationtrunc), root rule)
  // of the given leaves (by mode), inner nodes (the mode-1 product with the
  // node's own eigenvectors if m1, the products with the sons' if m23) and,
  // if root, the root
  struct ProjLabels { const char *factor, *leaf, *m1, *m2, *m3, *root; };
  auto emit_proj = [&](const std::vector<int>& modes, const std::vector<int>& inner, bool root,
                       const ProjLabels& L, bool m1, bool m23) {
    std::vector<GemmDesc> dp, du, d1, d2, d3;
    for (int mu : modes) {
      const int t = tr.leaf_node[mu];
      NodeBufs& b = O.nb[t];
      GemmDesc g = blank_desc();  // Pm = R^{-1} Qm
      g.A = b.Ri; g.sAm = b.K; g.sAk = 1;
      g.B = b.Qm; g.sBk = b.rcap; g.sBn = 1;
      g.C = b.Pm; g.sCm = b.rcap; g.sCn = 1;
      g.M = b.K; g.N = b.rcap; g.K = b.K;
      dp.push_back(g);
      GemmDesc u = blank_desc();  // U_new = W Pm
      u.nseg = S.n_in;
      for (int c = 0; c < S.n_in; ++c) {
        u.segA[c] = S.X[c]->leaf[mu];
        u.segAk[c] = S.X[c]->leaf_ld[mu];
        u.segBoff[c] = (int64_t)S.off[t][c] * b.rcap;
        u.segK[c] = S.X[c]->rank[t];
      }
      u.A = S.X[0]->leaf[mu]; u.sAm = 1;
      u.B = b.Pm; u.sBk = b.rcap; u.sBn = 1;
      u.C = need ? nullptr : out->leaf[mu]; u.sCm = 1; u.sCn = need ? 1 : out->leaf_ld[mu];
      u.M = (int)X[0].n[mu]; u.N = b.rcap;
      du.push_back(u);
    }
    for (int t : inner) {
      NodeBufs& b = O.nb[t];
      const int s1 = tr.son1[t], s2 = tr.son2[t];
      const int K1 = S.K[s1], K2 = S.K[s2];
      const int64_t w = (int64_t)K1 * K2;
      GemmDesc g = blank_desc();  // E1 = Qm_t^T M1(Qo)
      g.A = b.QmT; g.sAm = b.K; g.sAk = 1;
      g.B = b.Qo; g.sBk = w; g.sBn = 1;
      g.C = b.E1; g.sCm = w; g.sCn = 1;
      g.M = b.rcap; g.N = (int)w; g.K = b.K;
      d1.push_back(g);
      GemmDesc h = blank_desc();  // E2[a] = Qm_s1^T E1[a]
      h.A = O.nb[s1].QmT; h.sAm = K1; h.sAk = 1;
      h.B = b.E1; h.sBk = K2; h.sBn = 1; h.sBb = w;
      h.C = b.E2; h.sCm = K2; h.sCn = 1; h.sCb = (int64_t)O.nb[s1].rcap * K2;
      h.M = O.nb[s1].rcap; h.N = K2; h.K = K1; h.nbatch = b.rcap;
      d2.push_back(h);
      GemmDesc q = blank_desc();  // B_new = M12(E2) Qm_s2
      q.A = b.E2; q.sAm = K2; q.sAk = 1;
      q.B = O.nb[s2].QmT; q.sBk = 1; q.sBn = K2;
      q.C = need ? nullptr : out->transfer[t]; q.sCm = O.nb[s2].rcap; q.sCn = 1;
      q.M = b.rcap * O.nb[s1].rcap; q.N = O.nb[s2].rcap; q.K = K2;
      d3.push_back(q);
    }
    g_label = L.factor;
    add_gemm(P, dp, F64, F64, T, MATH_F64, GEMM_STORE, true, false);
    g_label = L.leaf;
    add_gemm(P, du, X[0].frame_dtype, T, need ? F64 : out->frame_dtype, fmath, GEMM_STORE, false, false, true);
    if (m1) {
      g_label = L.m1;
      add_gemm(P, d1, T, T, T, fmath, GEMM_STORE, true, false, true);
    }
    if (m23) {
      g_label = L.m2;
      add_gemm(P, d2, T, T, T, fmath, GEMM_STORE, true, false, true);
      g_label = L.m3;
      add_gemm(P, d3, T, T, need ? F64 : out->transfer_dtype, fmath, GEMM_STORE, true, true, true);
    }
    if (root) {
      g_label = L.root;
      // root: Qm_t1^T BDo Qm_t2
      const int t1 = tr.son1[0], t2 = tr.son2[0];
      const int K1r = S.K[t1], K2r = S.K[t2];
      std::vector<GemmDesc> r1, r2;
      GemmDesc g = blank_desc();
      g.A = O.nb[t1].Qm; g.sAm = 1; g.sAk = O.nb[t1].rcap;
      g.B = O.BDo; g.sBk = K2r; g.sBn = 1;
      g.C = O.T1; g.sCm = K2r; g.sCn = 1;
      g.M = O.nb[t1].rcap; g.N = K2r; g.K = K1r;
      r1.push_back(g);
      add_gemm(P, r1, F64, F64, F64, MATH_F64, GEMM_STORE, false, false);
      GemmDesc h = blank_desc();
      h.A = O.T1; h.sAm = K2r; h.sAk = 1;
      h.B = O.nb[t2].Qm; h.sBk = O.nb[t2].rcap; h.sBn = 1;
      h.C = need ? nullptr : out->transfer[0]; h.sCm = O.nb[t2].rcap; h.sCn = 1;
      h.M = O.nb[t1].rcap; h.N = O.nb[t2].rcap; h.K = K2r;
      // the result's root in units of 2^e_D (e_D goes to its scale): a
      // truncated tensor comes out with a root of norm below 1 however many
      // truncations it went through
      h.alpha_dev = &O.st->alpha_root;
      r2.push_back(h);
      add_gemm(P, r2, F64, F64, F64, MATH_F64, GEMM_STORE, true, false);
    }
  };
  // which projections can run with the upper eigenvectors alone
  std::vector<int> modes_up, modes_low, inner_up, inner_low;
  for (int mu = 0; mu < d; ++mu) (upper[tr.leaf_node[mu]] ? modes_up : modes_low).push_back(mu);
  for (int t = 1; t < nn; ++t) {
    if (tr.is_leaf(t)) continue;
    (upper[tr.son1[t]] && upper[tr.son2[t]] ? inner_up : inner_low).push_back(t);
  }
  const bool root_up = upper[tr.son1[0]] && upper[tr.son2[0]];
  const ProjLabels lab_low{"proj_leaf_factor", "proj_leaf", "proj_inner_mode1", "proj_inner_mode2",
                           "proj_inner_mode3", "proj_root"};
  const ProjLabels lab_up{"proj_leaf_factor_upper", "proj_leaf_upper", "proj_inner_mode1_upper",
                          "proj_inner_mode2_upper", "proj_inner_mode3_upper", "proj_root_upper"};
  // the mode-1 products of the inner nodes with lower sons need only their
  // own (upper) eigenvectors: they follow the upper projections on the
  // second stream, beside the lower eigensolver
  auto upper_part = [&](int dep) {
    if (!split || dep != Dmax - 2) return;
    add_sync(P, OP_FORK);
    g_stream = 1;
    emit_eig(up_nodes, "eig_upper");
    emit_rank_prep(up_nodes, "rank_select_upper", "proj_prep_upper");
    emit_proj(modes_up, inner_up, root_up, lab_up, true, true);
    const ProjLabels lab_side{"", "", "proj_inner_mode1_side", "", "", ""};
    emit_proj({}, inner_low, false, lab_side, true, false);
    g_stream = 0;
  };
  plan_gramians(P, tr, S.K, O.nb, O.BDo, O.st, Qo, T, upper_part);
  emit_eig(low_nodes, "eig");
  if (split) add_sync(P, OP_JOIN);
  emit_rank_prep(low_nodes, "rank_select", "proj_prep");
  emit_proj(modes_low, inner_low, !root_up, lab_low, !split, true);
  {
    g_label = "finish";
    StateRec r = blank_state(O.st);
    r.out_scale = reinterpret_cast<long long*>(out_scale); r.flags = flags; r.root_rank = out_ranks;
    r.add_eD = 1;
    add_state(P, OP_WRITESCALE, {r});
  }
  (void)tsz;
  if (need) *need = align256(A.off) + 256;
  if (used) *used = align256(A.off) + 256;
  return HT_OK;
}

ht_status ht_truncate_workspace(ht_context* ctx, const ht_desc* X, int32_t n_in, const ht_trunc_opts* opts,
                                size_t* bytes) {
  if (!bytes) return fail(HT_EINVAL, "bytes is NULL");
  if (!X) return fail(HT_EINVAL, "X is NULL");
  if (n_in < 1 || n_in > MAX_SEG) return fail(HT_EINVAL, "n_in must be in [1, 8]");
  Plan P;
  for (int c = 0; c < n_in; ++c) {
    ht_status s = check_desc(&X[c], "X[c]", false);
    if (s) return s;
  }
  // a dry run needs descriptors with data pointers; substitute placeholders
  std::vector<ht_desc> Xs(X, X + std::max(0, n_in));
  std::vector<std::vector<void*>> leaves(n_in), trans(n_in);
  std::vector<std::vector<int64_t>> lds(n_in);
  for (int c = 0; c < n_in; ++c) {
    leaves[c].assign(X[c].d, (void*)256);
    trans[c].assign(2 * X[c].d - 1, (void*)256);
    lds[c].assign(X[c].n, X[c].n + X[c].d);
    if (!X[c].leaf) Xs[c].leaf = leaves[c].data();
    if (!X[c].transfer) Xs[c].transfer = trans[c].data();
    if (!X[c].leaf_ld) Xs[c].leaf_ld = lds[c].data();
  }
  return build_truncate(ctx, Xs.data(), nullptr, n_in, opts, nullptr, nullptr, nullptr, nullptr, nullptr,
                        nullptr, P, bytes);
}

ht_status ht_truncate(ht_context* ctx, const ht_desc* X, const double* coef, int32_t n_in,
                      const ht_trunc_opts* opts, const ht_desc* out, int32_t* out_ranks,
                      int64_t* out_log2_scale, uint32_t* flags, double* out_sigma, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  size_t need = 0;
  ht_status st = ht_truncate_workspace(ctx, X, n_in, opts, &need);
  if (st) return st;
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(HT_EWORKSPACE, "workspace needs " + std::to_string(need) + " bytes, 256-byte aligned");
  HT_HIP(hipSetDevice(ctx->device));
  Plan P;
  st = build_truncate(ctx, X, coef, n_in, opts, out, out_ranks, out_log2_scale, flags, out_sigma, ws, P,
                      nullptr);
  if (st) return st;
  return run_plan(ctx, P, reinterpret_cast<hipStream_t>(stream));
}

ht_status ht_truncate_noalloc(ht_context* ctx, const ht_desc* X, const double* coef, int32_t n_in,
                              const ht_trunc_opts* opts, const ht_desc* out, int32_t* out_ranks,
                              int64_t* out_log2_scale, uint32_t* flags, double* out_sigma, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  if (ctx->device < 0 || ctx->device >= kNoAllocDevices)
    return fail(HT_EUNSUPPORTED, "ht_truncate_noalloc: device ids above 63 have no static scratch");
  NoAllocDevice& nd = g_noalloc[ctx->device];
  if (!nd.ptr) return fail(HT_EDEVICE, "ht_truncate_noalloc: the context was not set up on its device");
  size_t need = 0;
  ht_status st = ht_truncate_workspace(ctx, X, n_in, opts, &need);
  if (st) return st;
  const size_t ws_max = HT_NOALLOC_SCRATCH_BYTES - kNoAllocTableBytes;
  if (need > ws_max)
    return fail(HT_EWORKSPACE, "ht_truncate_noalloc: this truncation needs " + std::to_string(need) +
                                   " bytes of workspace; the static scratch holds " + std::to_string(ws_max));
  HT_HIP(hipSetDevice(ctx->device));
  char* base = reinterpret_cast<char*>(nd.ptr);
  Plan P;
  // one stream only: the second stream and its events would be created on first use
  st = build_truncate(ctx, X, coef, n_in, opts, out, out_ranks, out_log2_scale, flags, out_sigma,
                      base + kNoAllocTableBytes, P, nullptr, /*overlap=*/false);
  if (st) return st;
  if (P.table.size() > kNoAllocTableBytes)
    return fail(HT_EWORKSPACE, "ht_truncate_noalloc: launch tables of " + std::to_string(P.table.size()) +
                                   " bytes exceed the " + std::to_string(kNoAllocTableBytes) + " reserved");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(nd.mu);
  // Stream-ordered copy of the tables from host memory (pageable: the runtime
  // stages it before returning); skipped when the array already holds them.
  if (!P.table.empty() && P.table != nd.table) {
    nd.table = P.table;
    const hipError_t e = hipMemcpyAsync(base, nd.table.data(), nd.table.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      nd.table.clear();
      return fail(HT_EDEVICE, std::string("ht_truncate_noalloc: table copy: ") + hipGetErrorString(e));
    }
  }
  return launch_plan(ctx, P, base, s, /*allow_prof=*/false);
}

// ------------------------------------------------------------------ batched truncation
// The plans of the tensors of a batch, each with its own part of the
// workspace (need[c] bytes at offset off[c]), merged into one.
static ht_status build_truncate_batched(ht_context* ctx, int32_t count, const ht_desc* X, const int32_t* n_in,
                                        const double* coef, const ht_trunc_opts* opts, const ht_desc* out,
                                        int32_t* const* out_ranks, int64_t* out_scale, uint32_t* flags,
                                        double* const* out_sigma, void* ws, Plan& M, size_t* need,
                                        size_t* used = nullptr) {
  if (count < 1) return fail(HT_EINVAL, "count must be >= 1");
  if (!X || !n_in || !opts) return fail(HT_EINVAL, "X, n_in or opts is NULL");
  if (!need && (!out || !out_scale)) return fail(HT_EINVAL, "out or out_log2_scale is NULL");
  std::vector<Plan> plans(need ? 0 : count);
  size_t off = 0;
  int64_t first = 0;
  for (int c = 0; c < count; ++c) {
    if (n_in[c] < 1) return fail(HT_EINVAL, "n_in[" + std::to_string(c) + "] must be >= 1");
    const ht_desc* Xc = X + first;
    size_t nc = 0;
    ht_status st;
    if (need) {
      Plan dry;
      st = build_truncate(ctx, Xc, nullptr, n_in[c], &opts[c], nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                          dry, &nc);
    } else {
      // the problem's part of the workspace starts where the previous one ends
      char* wc = reinterpret_cast<char*>(ws) + off;
      st = build_truncate(ctx, Xc, coef ? coef + first : nullptr, n_in[c], &opts[c], &out[c],
                          out_ranks ? out_ranks[c] : nullptr, out_scale + c, flags ? flags + c : nullptr,
                          out_sigma ? out_sigma[c] : nullptr, wc, plans[c], nullptr, false, &nc);
    }
    if (st) return fail(st, "tensor " + std::to_string(c) + ": " + g_last_error);
    off += align256(nc);
    first += n_in[c];
  }
  if (need) {
    *need = off;
    return HT_OK;
  }
  if (used) *used = off;
  return merge_plans(plans, M);
}

ht_status ht_truncate_batched_workspace(ht_context* ctx, int32_t count, const ht_desc* X, const int32_t* n_in,
                                        const ht_trunc_opts* opts, size_t* bytes) {
  if (!bytes) return fail(HT_EINVAL, "bytes is NULL");
  if (count < 1 || !X || !n_in) return fail(HT_EINVAL, "count, X or n_in");
  int64_t tot = 0;
  for (int c = 0; c < count; ++c) {
    if (n_in[c] < 1) return fail(HT_EINVAL, "n_in[" + std::to_string(c) + "] must be >= 1");
    tot += n_in[c];
  }
  for (int64_t i = 0; i < tot; ++i) {
    ht_status s = check_desc(&X[i], "X[i]", false);
    if (s) return s;
  }
  // a dry run needs descriptors with data pointers; substitute placeholders
  std::vector<ht_desc> Xs(X, X + tot);
  std::vector<std::vector<void*>> leaves(tot), trans(tot);
  std::vector<std::vector<int64_t>> lds(tot);
  for (int64_t i = 0; i < tot; ++i) {
    leaves[i].assign(X[i].d, (void*)256);
    trans[i].assign(2 * X[i].d - 1, (void*)256);
    lds[i].assign(X[i].n, X[i].n + X[i].d);
    if (!X[i].leaf) Xs[i].leaf = leaves[i].data();
    if (!X[i].transfer) Xs[i].transfer = trans[i].data();
    if (!X[i].leaf_ld) Xs[i].leaf_ld = lds[i].data();
  }
  Plan M;
  return build_truncate_batched(ctx, count, Xs.data(), n_in, nullptr, opts, nullptr, nullptr, nullptr, nullptr,
                                nullptr, nullptr, M, bytes);
}

// Everything a batched plan depends on, as bytes: the contents of the
// descriptors (shapes, dtypes, data pointers, scales), coefficients, options,
// output pointers and the workspace.
extern "C++" {
static void sig_put(std::vector<unsigned char>& v, const void* p, size_t n) {
  const unsigned char* b = reinterpret_cast<const unsigned char*>(p);
  v.insert(v.end(), b, b + n);
}
template <typename T> static void sig_val(std::vector<unsigned char>& v, const T& x) { sig_put(v, &x, sizeof(T)); }
static void sig_desc(std::vector<unsigned char>& v, const ht_desc& x) {
  sig_val(v, x.d);
  sig_val(v, x.frame_dtype);
  sig_val(v, x.transfer_dtype);
  sig_val(v, x.log2_scale);
  const int nn = 2 * x.d - 1;
  sig_put(v, x.n, sizeof(int64_t) * x.d);
  sig_put(v, x.rank, sizeof(int32_t) * nn);
  sig_put(v, x.leaf, sizeof(void*) * x.d);
  sig_put(v, x.leaf_ld, sizeof(int64_t) * x.d);
  sig_put(v, x.transfer, sizeof(void*) * nn);
}
}  // extern "C++"

ht_status ht_truncate_batched(ht_context* ctx, int32_t count, const ht_desc* X, const int32_t* n_in,
                              const double* coef, const ht_trunc_opts* opts, const ht_desc* out,
                              int32_t* const* out_ranks, int64_t* out_log2_scale, uint32_t* flags,
                              double* const* out_sigma, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  if (count < 1 || !X || !n_in || !opts || !out) return fail(HT_EINVAL, "count, X, n_in, opts or out");
  int64_t tot = 0;
  for (int c = 0; c < count; ++c) tot += std::max(0, n_in[c]);
  for (int64_t i = 0; i < tot; ++i) {
    ht_status s = check_desc(&X[i], "X[i]");
    if (s) return s;
  }
  for (int c = 0; c < count; ++c) {
    ht_status s = check_desc(&out[c], "out[c]");
    if (s) return s;
  }
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return fail(HT_EWORKSPACE, "workspace must be 256-byte aligned");
  // a call with the same arguments as the previous one reuses its plan
  std::vector<unsigned char> sig;
  sig_val(sig, count);
  sig_put(sig, n_in, sizeof(int32_t) * count);
  for (int64_t i = 0; i < tot; ++i) {
    sig_desc(sig, X[i]);
    sig_val(sig, coef ? coef[i] : 1.0);
  }
  for (int c = 0; c < count; ++c) {
    const ht_trunc_opts& o = opts[c];
    sig_val(sig, o.mode); sig_val(sig, o.eps); sig_val(sig, o.eps_relative); sig_val(sig, o.max_rank);
    sig_val(sig, o.precision);
    if (o.mode == HT_RANK_FIXED && o.ranks) sig_put(sig, o.ranks, sizeof(int32_t) * (2 * out[c].d - 1));
    sig_desc(sig, out[c]);
    sig_val(sig, out_ranks ? out_ranks[c] : nullptr);
    sig_val(sig, out_sigma ? out_sigma[c] : nullptr);
  }
  sig_val(sig, out_log2_scale); sig_val(sig, flags); sig_val(sig, ws); sig_val(sig, ws_bytes);
  HT_HIP(hipSetDevice(ctx->device));
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->btable && ctx->bsig == sig) {
      Plan& B = ctx->bplan;
      void* t = ctx->btable;
      // launched outside the lock below would race a concurrent replacement;
      // the launches only enqueue, so holding the lock is cheap
      return launch_plan(ctx, B, t, reinterpret_cast<hipStream_t>(stream));
    }
  }
  // the plans are built once, each problem taking the next part of the
  // workspace; nothing is launched unless the whole of it fits
  Plan M;
  size_t need = 0;
  ht_status st = build_truncate_batched(ctx, count, X, n_in, coef, opts, out, out_ranks, out_log2_scale, flags,
                                        out_sigma, ws, M, nullptr, &need);
  if (st) return st;
  if (ws_bytes < need)
    return fail(HT_EWORKSPACE, "workspace needs " + std::to_string(need) + " bytes, 256-byte aligned");
  void* table = nullptr;
  if (!M.table.empty()) {
    HT_HIP(hipMalloc(&table, M.table.size()));
    const hipError_t e = hipMemcpy(table, M.table.data(), M.table.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(table);
      return fail(HT_EDEVICE, std::string("batch table upload: ") + hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->btable) {
    HT_HIP(hipDeviceSynchronize());   // the previous table may still be read by queued launches
    (void)hipFree(ctx->btable);
  }
  M.table.clear();
  M.table.shrink_to_fit();
  ctx->bsig.swap(sig);
  ctx->bplan = std::move(M);
  ctx->btable = table;
  return launch_plan(ctx, ctx->bplan, table, reinterpret_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ orthogonalisation
static ht_status build_orth(const ht_desc* X, int precision, int64_t* out_scale, uint32_t* flags, void* ws,
                            Plan& P, size_t* need) {
  if (precision != HT_PREC_FP64 && precision != HT_PREC_MIXED) return fail(HT_EINVAL, "bad precision");
  SumInfo S;
  ht_status st = sum_info(X, nullptr, 1, S);
  if (st) return st;
  Tree tr(X->d);
  for (int mu = 0; mu < X->d; ++mu)
    if (X->n[mu] < X->rank[tr.leaf_node[mu]]) return fail(HT_EUNSUPPORTED, "orthogonalisation needs n_mu >= k_mu");
  if (!need && !out_scale) return fail(HT_EINVAL, "out_log2_scale is NULL");
  Arena A(ws);
  OrthOut O;
  plan_orth(P, tr, S, precision, A, O, {}, false, nullptr, X);
  // leaves: Q = W R^{-1} into the frame buffer (via the sweep-2 temporary)
  std::vector<GemmDesc> dq;
  for (int mu = 0; mu < X->d; ++mu) {
    const int t = tr.leaf_node[mu];
    GemmDesc g = blank_desc();
    g.A = X->leaf[mu]; g.sAm = 1; g.sAk = X->leaf_ld[mu];
    g.B = O.nb[t].Ri; g.sBk = S.K[t]; g.sBn = 1;
    g.C = O.nb[t].Y; g.sCm = 1; g.sCn = X->n[mu];
    g.M = (int)X->n[mu]; g.N = S.K[t]; g.K = S.K[t];
    dq.push_back(g);
  }
  add_gemm(P, dq, X->frame_dtype, F64, F64, MATH_F64, GEMM_STORE, false, false);
  {
    std::vector<CopyRec> cr;
    for (int mu = 0; mu < X->d; ++mu) {
      const int t = tr.leaf_node[mu];
      CopyRec q;
      std::memset(&q, 0, sizeof(q));
      q.src = O.nb[t].Y; q.tsrc = F64; q.dst = X->leaf[mu]; q.tdst = X->frame_dtype;
      q.n0 = 1; q.n1 = X->n[mu]; q.n2 = S.K[t]; q.s1 = 1; q.s2 = X->n[mu]; q.d1 = 1; q.d2 = X->leaf_ld[mu];
      q.alpha = 1.0;
      cr.push_back(q);
    }
    add_copies(P, cr);
  }
  {
    StateRec r = blank_state(O.st);
    r.out_scale = reinterpret_cast<long long*>(out_scale); r.flags = flags;
    add_state(P, OP_WRITESCALE, {r});
  }
  if (need) *need = align256(A.off) + 256;
  return HT_OK;
}

ht_status ht_orthogonalize_workspace(ht_context* ctx, const ht_desc* X, int32_t precision, size_t* bytes) {
  (void)ctx;
  if (!bytes) return fail(HT_EINVAL, "NULL argument");
  ht_status s = check_desc(X, "X", false);
  if (s) return s;
  std::vector<void*> lv(X->d, (void*)256), tv(2 * X->d - 1, (void*)256);
  std::vector<int64_t> ld(X->n, X->n + X->d);
  ht_desc Y = *X;
  if (!Y.leaf) Y.leaf = lv.data();
  if (!Y.transfer) Y.transfer = tv.data();
  if (!Y.leaf_ld) Y.leaf_ld = ld.data();
  Plan P;
  return build_orth(&Y, precision, nullptr, nullptr, nullptr, P, bytes);
}

ht_status ht_orthogonalize(ht_context* ctx, const ht_desc* X, int32_t precision, int64_t* out_log2_scale,
                           uint32_t* flags, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  size_t need = 0;
  ht_status st = ht_orthogonalize_workspace(ctx, X, precision, &need);
  if (st) return st;
  st = check_desc(X, "X");
  if (st) return st;
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(HT_EWORKSPACE, "workspace needs " + std::to_string(need) + " bytes, 256-byte aligned");
  HT_HIP(hipSetDevice(ctx->device));
  Plan P;
  st = build_orth(X, precision, out_log2_scale, flags, ws, P, nullptr);
  if (st) return st;
  return run_plan(ctx, P, reinterpret_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ Gramians of an orthogonal tensor
static ht_status build_gram(const ht_desc* X, double* const* bhat, double* const* sigma, int64_t* out_units,
                            void* ws, Plan& P, size_t* need) {
  Tree tr(X->d);
  const int nn = tr.nn;
  std::vector<int> K(nn, 1);
  for (int t = 1; t < nn; ++t) {
    K[t] = X->rank[t];
    if (K[t] > KMAX) return fail(HT_EUNSUPPORTED, "rank above 128");
  }
  if (!need) {
    if (!bhat) return fail(HT_EINVAL, "bhat is NULL");
    for (int t = 1; t < nn; ++t)
      if (!bhat[t]) return fail(HT_EINVAL, "bhat[t] is NULL");
  }
  Arena A(ws);
  std::vector<NodeBufs> nb(nn);
  size_t z0 = A.off;
  for (int t = 1; t < nn; ++t) {
    nb[t].K = K[t];
    nb[t].Bh = need ? (double*)A.take((size_t)K[t] * K[t] * 8) : bhat[t];
  }
  if (!need) {
    // the Gramians are accumulated atomically into the caller's arrays: clear them
  }
  GlobalState* st = (GlobalState*)A.take(sizeof(GlobalState));
  for (int t = 1; t < nn; ++t) {
    if (tr.is_leaf(t)) continue;
    nb[t].C = (double*)A.take((size_t)K[t] * K[tr.son1[t]] * K[tr.son2[t]] * 8);
  }
  const bool want_sigma = sigma != nullptr;
  for (int t = 1; t < nn && want_sigma; ++t) {
    nb[t].Q = (double*)A.take((size_t)K[t] * K[t] * 8);
    nb[t].lam = (double*)A.take((size_t)K[t] * 8);
    nb[t].scratch = (double*)A.take(eig_scratch_doubles(K[t]) * 8);
  }
  {
    StateRec r = blank_state(st);
    r.scale0 = X->log2_scale;
    add_state(P, OP_SETSTATE, {r});
  }
  if (!need) {
    std::vector<FillRec> fr;
    for (int t = 1; t < nn; ++t) fr.push_back(FillRec{nb[t].Bh, (size_t)K[t] * K[t] * 8});
    add_fills(P, fr);
  }
  std::vector<const void*> Qo(nn, nullptr);
  for (int t = 1; t < nn; ++t) Qo[t] = X->transfer ? X->transfer[t] : nullptr;
  plan_gramians(P, tr, K, nb, (const double*)X->transfer[0], st, Qo, X->transfer_dtype);
  if (want_sigma) {
    std::vector<SmallArgs> sa;
    std::vector<double*> sp;
    for (int t = 1; t < nn; ++t) {
      SmallArgs a;
      std::memset(&a, 0, sizeof(a));
      a.K = K[t]; a.node = t; a.Q = nb[t].Q; a.lam = nb[t].lam; a.scratch = nb[t].scratch; a.Bh = nb[t].Bh;
      sa.push_back(a);
      sp.push_back(sigma[t]);
    }
    add_small(P, OP_EIG, sa);
    P.ops.back().p0 = st;
    add_small(P, OP_SIGMA, sa);
    P.ops.back().bytes = put(P, sp);
  }
  if (out_units) {
    StateRec r = blank_state(st);
    r.out_scale = reinterpret_cast<long long*>(out_units); r.add_eD = 1;
    add_state(P, OP_WRITESCALE, {r});
  }
  if (need) *need = align256(A.off) + 256;
  (void)z0;
  return HT_OK;
}

ht_status ht_gramians_workspace(ht_context* ctx, const ht_desc* X, size_t* bytes) {
  (void)ctx;
  if (!bytes) return fail(HT_EINVAL, "NULL argument");
  ht_status s = check_desc(X, "X", false);
  if (s) return s;
  std::vector<void*> tv(2 * X->d - 1, (void*)256);
  ht_desc Y = *X;
  if (!Y.transfer) Y.transfer = tv.data();
  Plan P;
  // sized with the optional eigensolver buffers (sigma requested)
  static double* const placeholder[1] = {nullptr};
  return build_gram(&Y, nullptr, placeholder, nullptr, nullptr, P, bytes);
}

ht_status ht_gramians(ht_context* ctx, const ht_desc* X, double* const* bhat, double* const* sigma,
                      int64_t* out_log2_units, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  size_t need = 0;
  ht_status st = ht_gramians_workspace(ctx, X, &need);
  if (st) return st;
  st = check_desc(X, "X");
  if (st) return st;
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(HT_EWORKSPACE, "workspace needs " + std::to_string(need) + " bytes, 256-byte aligned");
  HT_HIP(hipSetDevice(ctx->device));
  Plan P;
  st = build_gram(X, bhat, sigma, out_log2_units, ws, P, nullptr);
  if (st) return st;
  return run_plan(ctx, P, reinterpret_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ inner product (Section 3.2)
// A descriptor whose NULL data arrays are replaced by placeholder addresses
// (workspace queries plan with fake pointers and never dereference them).
struct Placeholder {
  ht_desc d{};
  std::vector<void*> leaves, trans;
  std::vector<int64_t> lds;
  explicit Placeholder(const ht_desc* X) : d(*X) {
    leaves.assign(X->d, (void*)256);
    trans.assign(2 * X->d - 1, (void*)256);
    lds.assign(X->n, X->n + X->d);
    if (!X->leaf) d.leaf = leaves.data();
    if (!X->transfer) d.transfer = trans.data();
    if (!X->leaf_ld) d.leaf_ld = lds.data();
  }
};

// <X, Y> by Definition (phi), bottom-up one tree level per launch:
//   leaves        Phi_mu = U_mu^T V_mu                      (split-K products)
//   inner nodes   eq. (defphi): T1 = B_t x_2 Phi_s1^T, T2 = T1 x_3 Phi_s2^T,
//                 Phi_t = M_1(T2) M_1(F_t)^T
//   root          Phi_D = sum_{b,c} B_D[b,c] (Phi_t1 F_D Phi_t2^T)[b,c]
// (B: transfer tensors of X, F: of Y).  After each level every Phi_t is
// divided by a power of two and the exponents are summed up the tree, so
// the result is out_val * 2^out_log2 with 0.5 <= |out_val| < 1 (or 0).
static ht_status build_inner(const ht_desc* X, const ht_desc* Y, double* out_val, int64_t* out_log2,
                             uint32_t* flags, void* ws, Plan& P, size_t* need) {
  ht_status st;
  if ((st = check_desc(X, "X")) || (st = check_desc(Y, "Y"))) return st;
  if (X->d != Y->d) return fail(HT_ESHAPE, "X and Y must share d");
  const int d = X->d;
  for (int mu = 0; mu < d; ++mu)
    if (X->n[mu] != Y->n[mu]) return fail(HT_ESHAPE, "X and Y must share n");
  Tree tr(d);
  const int nn = tr.nn;
  for (int t = 1; t < nn; ++t)
    if (X->rank[t] > KMAX || Y->rank[t] > KMAX) return fail(HT_EUNSUPPORTED, "ranks above 128");
  Arena A(ws);
  // zero region: the split-K targets Phi_t (k^X_t x k^Y_t) and the root value
  std::vector<double*> phi(nn, nullptr);
  const size_t z0 = align256(A.off);
  A.off = z0;
  for (int t = 1; t < nn; ++t) phi[t] = (double*)A.take((size_t)X->rank[t] * Y->rank[t] * 8);
  phi[0] = (double*)A.take(8);
  const size_t zbytes = A.off - z0;
  void* zptr = A.base ? A.base + z0 : nullptr;
  reg(zptr, zbytes, "zero region");
  std::vector<long long*> E(nn, nullptr);
  for (int t = 0; t < nn; ++t) E[t] = (long long*)A.take(8);
  // per-level temporaries, reused level after level (one stream)
  size_t t1max = 0, t2max = 0;
  const int H = tr.height[0];
  for (int h = 1; h < H; ++h) {
    size_t a = 0, b = 0;
    for (int t = 1; t < nn; ++t) {
      if (tr.is_leaf(t) || tr.height[t] != h) continue;
      const int s1 = tr.son1[t], s2 = tr.son2[t];
      a += (size_t)X->rank[t] * Y->rank[s1] * X->rank[s2];
      b += (size_t)X->rank[t] * Y->rank[s1] * Y->rank[s2];
    }
    t1max = std::max(t1max, a);
    t2max = std::max(t2max, b);
  }
  double* T1 = (double*)A.take(std::max<size_t>(t1max, 1) * 8);
  double* T2 = (double*)A.take(std::max<size_t>(t2max, 1) * 8);
  const int r1 = tr.son1[0], r2 = tr.son2[0];
  double* W1 = (double*)A.take((size_t)X->rank[r1] * Y->rank[r2] * 8);
  double* W2 = (double*)A.take((size_t)X->rank[r1] * X->rank[r2] * 8);
  if (need) *need = align256(A.off) + 256;
  if (!ws) return HT_OK;

  const int fX = X->frame_dtype, fY = Y->frame_dtype, tX = X->transfer_dtype, tY = Y->transfer_dtype;
  g_label = "inner_setup";
  add_fill(P, zptr, zbytes);
  // leaves
  g_label = "inner_leaf";
  {
    std::vector<GemmDesc> dl;
    std::vector<PhiRec> pr;
    for (int mu = 0; mu < d; ++mu) {
      const int t = tr.leaf_node[mu];
      GemmDesc g = blank_desc();
      g.A = X->leaf[mu]; g.sAm = X->leaf_ld[mu]; g.sAk = 1;
      g.B = Y->leaf[mu]; g.sBk = 1; g.sBn = Y->leaf_ld[mu];
      g.C = phi[t]; g.sCm = Y->rank[t]; g.sCn = 1;
      g.M = X->rank[t]; g.N = Y->rank[t]; g.K = (int)X->n[mu];
      dl.push_back(g);
      PhiRec r = blank_phi();
      r.P = phi[t]; r.n = (int64_t)X->rank[t] * Y->rank[t]; r.E = E[t]; r.flags = flags;
      pr.push_back(r);
    }
    add_gemm(P, dl, fX, fY, F64, MATH_F64, GEMM_ATOMIC, true, true);
    add_phi(P, pr);
  }
  // inner nodes by height
  for (int h = 1; h < H; ++h) {
    std::vector<GemmDesc> d1, d2, d3;
    std::vector<PhiRec> pr;
    size_t o1 = 0, o2 = 0;
    for (int t = 1; t < nn; ++t) {
      if (tr.is_leaf(t) || tr.height[t] != h) continue;
      const int s1 = tr.son1[t], s2 = tr.son2[t];
      const int a = X->rank[t], b = X->rank[s1], c = X->rank[s2];
      const int f = Y->rank[t], dd = Y->rank[s1], e = Y->rank[s2];
      double* t1 = T1 + o1;
      double* t2 = T2 + o2;
      o1 += (size_t)a * dd * c;
      o2 += (size_t)a * dd * e;
      // T1[a][d][c] = sum_b Phi_s1[b][d] B[a][b][c]   (one product per a)
      GemmDesc g = blank_desc();
      g.A = phi[s1]; g.sAm = 1; g.sAk = dd;
      g.B = X->transfer[t]; g.sBk = c; g.sBn = 1; g.sBb = (int64_t)b * c;
      g.C = t1; g.sCm = c; g.sCn = 1; g.sCb = (int64_t)dd * c;
      g.M = dd; g.N = c; g.K = b; g.nbatch = a;
      d1.push_back(g);
      // T2[(a,d)][e] = sum_c T1[(a,d)][c] Phi_s2[c][e]
      GemmDesc q = blank_desc();
      q.A = t1; q.sAm = c; q.sAk = 1;
      q.B = phi[s2]; q.sBk = e; q.sBn = 1;
      q.C = t2; q.sCm = e; q.sCn = 1;
      q.M = a * dd; q.N = e; q.K = c;
      d2.push_back(q);
      // Phi_t[a][f] = sum_{(d,e)} T2[a][(d,e)] F[f][(d,e)]
      GemmDesc r = blank_desc();
      r.A = t2; r.sAm = (int64_t)dd * e; r.sAk = 1;
      r.B = Y->transfer[t]; r.sBk = 1; r.sBn = (int64_t)dd * e;
      r.C = phi[t]; r.sCm = f; r.sCn = 1;
      r.M = a; r.N = f; r.K = dd * e;
      d3.push_back(r);
      PhiRec pz = blank_phi();
      pz.P = phi[t]; pz.n = (int64_t)a * f; pz.E = E[t]; pz.E1 = E[s1]; pz.E2 = E[s2]; pz.flags = flags;
      pr.push_back(pz);
    }
    if (pr.empty()) continue;
    g_label = "inner_mode2";
    add_gemm(P, d1, F64, tX, F64, MATH_F64, GEMM_STORE, false, false);
    g_label = "inner_mode3";
    add_gemm(P, d2, F64, F64, F64, MATH_F64, GEMM_STORE, true, false);
    g_label = "inner_contract";
    add_gemm(P, d3, F64, tY, F64, MATH_F64, GEMM_ATOMIC, true, true);
    add_phi(P, pr);
  }
  // root: W1 = Phi_t1 F_D, W2 = W1 Phi_t2^T, Phi_D = <B_D, W2>
  g_label = "inner_root";
  {
    const int b = X->rank[r1], c = X->rank[r2], dd = Y->rank[r1], e = Y->rank[r2];
    GemmDesc g = blank_desc();
    g.A = phi[r1]; g.sAm = dd; g.sAk = 1;
    g.B = Y->transfer[0]; g.sBk = e; g.sBn = 1;
    g.C = W1; g.sCm = e; g.sCn = 1;
    g.M = b; g.N = e; g.K = dd;
    add_gemm(P, {g}, F64, F64, F64, MATH_F64, GEMM_STORE, true, false);
    GemmDesc q = blank_desc();
    q.A = W1; q.sAm = e; q.sAk = 1;
    q.B = phi[r2]; q.sBk = 1; q.sBn = e;
    q.C = W2; q.sCm = c; q.sCn = 1;
    q.M = b; q.N = c; q.K = e;
    add_gemm(P, {q}, F64, F64, F64, MATH_F64, GEMM_STORE, true, true);
    GemmDesc r = blank_desc();
    r.A = X->transfer[0]; r.sAm = (int64_t)b * c; r.sAk = 1;
    r.B = W2; r.sBk = 1; r.sBn = (int64_t)b * c;
    r.C = phi[0]; r.sCm = 1; r.sCn = 1;
    r.M = 1; r.N = 1; r.K = b * c;
    add_gemm(P, {r}, F64, F64, F64, MATH_F64, GEMM_ATOMIC, true, true);
    PhiRec pz = blank_phi();
    pz.P = phi[0]; pz.n = 1; pz.E = E[0]; pz.E1 = E[r1]; pz.E2 = E[r2];
    pz.out_val = out_val; pz.out_log2 = reinterpret_cast<long long*>(out_log2);
    pz.add = X->log2_scale + Y->log2_scale; pz.flags = flags; pz.mode = 1;
    add_phi(P, {pz});
  }
  return HT_OK;
}

// ||sum_c coef_c X_c|| as out_val * 2^out_log2: the lazy sum is orthogonalised
// bottom-up (Section 3.4, the R factors only) and the norm of an orthogonal
// HT tensor is the Frobenius norm of its root matrix.  With X_1 - X_2 this is
// the difference norm, free of the cancellation of <X,X> - 2<X,Y> + <Y,Y>.
static ht_status build_norm(const ht_desc* X, const double* coef, int32_t n_in, double* out_val,
                            int64_t* out_log2, uint32_t* flags, void* ws, Plan& P, size_t* need) {
  if (!X) return fail(HT_EINVAL, "X is NULL");
  SumInfo S;
  ht_status st = sum_info(X, coef, n_in, S);
  if (st) return st;
  Tree tr(X[0].d);
  Arena A(ws);
  OrthOut O;
  plan_orth(P, tr, S, HT_PREC_FP64, A, O, {}, false, nullptr, nullptr, false, /*form_qo=*/false);
  if (need) *need = align256(A.off) + 256;
  if (!ws) return HT_OK;
  g_label = "norm_root";
  PhiRec r = blank_phi();
  r.P = O.BDo; r.n = (int64_t)S.K[tr.son1[0]] * S.K[tr.son2[0]];
  r.out_val = out_val; r.out_log2 = reinterpret_cast<long long*>(out_log2);
  r.add_dev = &O.st->log2_scale; r.flags = flags; r.mode = 2;
  add_phi(P, {r});
  if (flags) {
    g_label = "finish";
    StateRec w = blank_state(O.st);
    w.flags = flags;
    add_state(P, OP_WRITESCALE, {w});
  }
  return HT_OK;
}

ht_status ht_inner_workspace(ht_context* ctx, const ht_desc* X, const ht_desc* Y, size_t* bytes) {
  (void)ctx;
  if (!bytes) return fail(HT_EINVAL, "bytes is NULL");
  if (!X || !Y) return fail(HT_EINVAL, "X or Y is NULL");
  ht_status st;
  if ((st = check_desc(X, "X", false)) || (st = check_desc(Y, "Y", false))) return st;
  Placeholder px(X), py(Y);
  Plan P;
  return build_inner(&px.d, &py.d, nullptr, nullptr, nullptr, nullptr, P, bytes);
}

ht_status ht_inner(ht_context* ctx, const ht_desc* X, const ht_desc* Y, double* out_val, int64_t* out_log2,
                   uint32_t* flags, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  if (!out_val || !out_log2) return fail(HT_EINVAL, "out_val and out_log2 are required");
  size_t need = 0;
  ht_status st = ht_inner_workspace(ctx, X, Y, &need);
  if (st) return st;
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(HT_EWORKSPACE, "workspace needs " + std::to_string(need) + " bytes, 256-byte aligned");
  HT_HIP(hipSetDevice(ctx->device));
  Plan P;
  st = build_inner(X, Y, out_val, out_log2, flags, ws, P, nullptr);
  if (st) return st;
  return run_plan(ctx, P, reinterpret_cast<hipStream_t>(stream));
}

ht_status ht_norm_workspace(ht_context* ctx, const ht_desc* X, int32_t n_in, size_t* bytes) {
  (void)ctx;
  if (!bytes) return fail(HT_EINVAL, "bytes is NULL");
  if (!X) return fail(HT_EINVAL, "X is NULL");
  if (n_in < 1 || n_in > MAX_SEG) return fail(HT_EINVAL, "n_in must be in [1, 8]");
  std::vector<Placeholder> ph;
  ph.reserve(n_in);
  std::vector<ht_desc> xs;
  for (int c = 0; c < n_in; ++c) {
    ht_status s = check_desc(&X[c], "X[c]", false);
    if (s) return s;
    ph.emplace_back(&X[c]);
    xs.push_back(ph.back().d);
  }
  Plan P;
  return build_norm(xs.data(), nullptr, n_in, nullptr, nullptr, nullptr, nullptr, P, bytes);
}

ht_status ht_norm(ht_context* ctx, const ht_desc* X, const double* coef, int32_t n_in, double* out_val,
                  int64_t* out_log2, uint32_t* flags, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  if (!out_val || !out_log2) return fail(HT_EINVAL, "out_val and out_log2 are required");
  size_t need = 0;
  ht_status st = ht_norm_workspace(ctx, X, n_in, &need);
  if (st) return st;
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(HT_EWORKSPACE, "workspace needs " + std::to_string(need) + " bytes, 256-byte aligned");
  HT_HIP(hipSetDevice(ctx->device));
  Plan P;
  st = build_norm(X, coef, n_in, out_val, out_log2, flags, ws, P, nullptr);
  if (st) return st;
  return run_plan(ctx, P, reinterpret_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ operator application (Section 3.6)
// C = L A by Lemma (operator): leaf frames V_mu[:, r k_mu + l] = W_{mu,r} U_mu[:, l]
// (one batched product per leaf, a batch entry per operator rank r), and
// every transfer tensor F_t = H_t (x) B_t (the operator index slowest).
static ht_status build_apply(const ht_desc* L, const ht_desc* A, const ht_desc* C, Plan& P) {
  ht_status st;
  if ((st = check_desc(L, "L")) || (st = check_desc(A, "A")) || (st = check_desc(C, "C"))) return st;
  const int d = A->d;
  if (L->d != d || C->d != d) return fail(HT_ESHAPE, "L, A and C must share d");
  Tree tr(d);
  for (int mu = 0; mu < d; ++mu) {
    const int64_t n = A->n[mu];
    if (L->n[mu] != n * n) return fail(HT_ESHAPE, "operator frames must have n_mu^2 rows (square operators)");
    if (C->n[mu] != n) return fail(HT_ESHAPE, "C must have the mode sizes of A");
  }
  for (int t = 1; t < tr.nn; ++t)
    if (C->rank[t] != L->rank[t] * A->rank[t])
      return fail(HT_ESHAPE, "C's ranks must be the products of L's and A's (node " + std::to_string(t) + ")");
  g_label = "apply_leaf";
  std::vector<GemmDesc> dl;
  for (int mu = 0; mu < d; ++mu) {
    const int t = tr.leaf_node[mu];
    const int64_t n = A->n[mu];
    GemmDesc g = blank_desc();
    g.A = L->leaf[mu]; g.sAm = n; g.sAk = 1; g.sAb = L->leaf_ld[mu];       // W_{mu,r}[j][i]
    g.B = A->leaf[mu]; g.sBk = 1; g.sBn = A->leaf_ld[mu];                  // U_mu[i][l]
    g.C = C->leaf[mu]; g.sCm = 1; g.sCn = C->leaf_ld[mu];                  // V_mu[j][r k + l]
    g.sCb = (int64_t)A->rank[t] * C->leaf_ld[mu];
    g.M = (int)n; g.N = A->rank[t]; g.K = (int)n; g.nbatch = L->rank[t];
    dl.push_back(g);
  }
  add_gemm(P, dl, L->frame_dtype, A->frame_dtype, C->frame_dtype, MATH_F64, GEMM_STORE, true, true);
  g_label = "apply_transfer";
  std::vector<KronRec> kr;
  for (int t = 0; t < tr.nn; ++t) {
    if (tr.is_leaf(t)) continue;
    const int s1 = tr.son1[t], s2 = tr.son2[t];
    KronRec r;
    std::memset(&r, 0, sizeof(r));
    r.H = L->transfer[t]; r.B = A->transfer[t]; r.F = C->transfer[t];
    r.tH = t == 0 ? F64 : L->transfer_dtype;
    r.tB = t == 0 ? F64 : A->transfer_dtype;
    r.tF = t == 0 ? F64 : C->transfer_dtype;
    r.P = t == 0 ? 1 : L->rank[t]; r.Q = L->rank[s1]; r.R = L->rank[s2];
    r.I = t == 0 ? 1 : A->rank[t]; r.J = A->rank[s1]; r.L = A->rank[s2];
    kr.push_back(r);
  }
  add_kron(P, kr);
  return HT_OK;
}

ht_status ht_apply(ht_context* ctx, const ht_desc* L, const ht_desc* A, const ht_desc* C, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  HT_HIP(hipSetDevice(ctx->device));
  Plan P;
  ht_status st = build_apply(L, A, C, P);
  if (st) return st;
  return run_plan(ctx, P, reinterpret_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ entries
static size_t entries_chunk(const ht_desc* X, int64_t m, size_t* per_index) {
  Tree tr(X->d);
  size_t per = 0;
  for (int t = 0; t < tr.nn; ++t) per += (size_t)(t == 0 ? 1 : X->rank[t]) * 8 + 4 + 16;
  *per_index = per;
  const size_t cap = (size_t)1 << 31;
  size_t ch = std::max<size_t>(1024, cap / per);
  return (size_t)std::min<int64_t>(m, (int64_t)ch);
}

static ht_status build_entries(const ht_desc* X, int64_t m, const int32_t* idx, double* out, void* ws, Plan& P,
                               size_t* need) {
  Tree tr(X->d);
  const int nn = tr.nn, d = X->d;
  for (int t = 1; t < nn; ++t)
    if (X->rank[t] > 4096) return fail(HT_EUNSUPPORTED, "rank too large for entries");
  size_t per = 0;
  const int64_t ch = m > 0 ? (int64_t)entries_chunk(X, m, &per) : 0;
  Arena A(ws);
  std::vector<double*> rows(nn);
  std::vector<int32_t*> expo(nn);
  for (int t = 0; t < nn; ++t) {
    const int k = t == 0 ? 1 : X->rank[t];
    rows[t] = (double*)A.take((size_t)std::max<int64_t>(ch, 1) * k * 8);
    expo[t] = (int32_t*)A.take((size_t)std::max<int64_t>(ch, 1) * 4);
  }
  if (need) {
    *need = align256(A.off) + 256;
    return HT_OK;
  }
  const int H = tr.height[0];
  for (int64_t c0 = 0; c0 < m; c0 += ch) {
    const int64_t mc = std::min<int64_t>(ch, m - c0);
    // leaves
    std::vector<EntryNode> lv;
    for (int mu = 0; mu < d; ++mu) {
      const int t = tr.leaf_node[mu];
      EntryNode e;
      std::memset(&e, 0, sizeof(e));
      e.k = X->rank[t]; e.mode = mu; e.tdtype = X->frame_dtype; e.U = X->leaf[mu]; e.ld = X->leaf_ld[mu];
      e.rows = rows[t]; e.expo = expo[t];
      lv.push_back(e);
    }
    Op g; g.kind = OP_EGATHER; g.toff = put(P, lv); g.count = (int)lv.size(); g.c[0] = mc;
    g.p0 = const_cast<int32_t*>(idx + c0 * d); g.i0 = d;
    P.ops.push_back(g);
    Op nrm; nrm.kind = OP_ENORM; nrm.toff = g.toff; nrm.count = g.count; nrm.c[0] = mc;
    P.ops.push_back(nrm);
    for (int h = 1; h <= H; ++h) {
      std::vector<GemmDesc> ds;
      std::vector<EntryNode> en;
      for (int t = 0; t < nn; ++t) {
        if (tr.is_leaf(t) || tr.height[t] != h) continue;
        const int s1 = tr.son1[t], s2 = tr.son2[t];
        const int k1 = X->rank[s1], k2 = X->rank[s2], kt = t == 0 ? 1 : X->rank[t];
        GemmDesc q = blank_desc();
        q.kr = 1; q.krK2 = k2; q.krY1 = rows[s1]; q.krY2 = rows[s2]; q.krld1 = k1; q.krld2 = k2;
        q.A = rows[s1]; q.sAm = 0; q.sAk = 1;
        q.B = X->transfer[t]; q.sBk = 1; q.sBn = (int64_t)k1 * k2;
        q.C = rows[t]; q.sCm = kt; q.sCn = 1;
        q.M = (int)mc; q.N = kt; q.K = k1 * k2;
        ds.push_back(q);
        EntryNode e;
        std::memset(&e, 0, sizeof(e));
        e.k = kt; e.rows = rows[t]; e.expo = expo[t]; e.expo1 = expo[s1]; e.expo2 = expo[s2];
        en.push_back(e);
      }
      if (ds.empty()) continue;
      // the root matrix is float64; inner transfer tensors have transfer_dtype
      std::vector<GemmDesc> dr, di;
      for (auto& q : ds) (q.N == 1 && q.B == X->transfer[0] ? dr : di).push_back(q);
      add_gemm(P, di, F64, X->transfer_dtype, F64, MATH_F64, GEMM_STORE, true, true);
      add_gemm(P, dr, F64, F64, F64, MATH_F64, GEMM_STORE, true, true);
      Op n2; n2.kind = OP_ENORM; n2.toff = put(P, en); n2.count = (int)en.size(); n2.c[0] = mc;
      P.ops.push_back(n2);
    }
    Op f; f.kind = OP_EFINISH; f.p0 = rows[0]; f.p1 = expo[0]; f.p2 = out + c0; f.c[0] = mc;
    f.scale0 = X->log2_scale;
    P.ops.push_back(f);
  }
  return HT_OK;
}

ht_status ht_entries_workspace(ht_context* ctx, const ht_desc* X, int64_t m, size_t* bytes) {
  (void)ctx;
  if (!bytes) return fail(HT_EINVAL, "NULL argument");
  if (m < 0) return fail(HT_EINVAL, "m must be >= 0");
  ht_status s = check_desc(X, "X", false);
  if (s) return s;
  Plan P;
  return build_entries(X, m, nullptr, nullptr, nullptr, P, bytes);
}

ht_status ht_entries(ht_context* ctx, const ht_desc* X, int64_t m, const int32_t* idx, double* out, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  size_t need = 0;
  ht_status st = ht_entries_workspace(ctx, X, m, &need);
  if (st) return st;
  st = check_desc(X, "X");
  if (st) return st;
  if (m == 0) return HT_OK;
  if (!idx || !out) return fail(HT_EINVAL, "idx or out is NULL");
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(HT_EWORKSPACE, "workspace needs " + std::to_string(need) + " bytes, 256-byte aligned");
  HT_HIP(hipSetDevice(ctx->device));
  Plan P;
  st = build_entries(X, m, idx, out, ws, P, nullptr);
  if (st) return st;
  return run_plan(ctx, P, reinterpret_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ sum (Lemma (sum))
ht_status ht_add(ht_context* ctx, double alpha, const ht_desc* A, double beta, const ht_desc* C, const ht_desc* S,
                 int64_t* out_log2_scale, void* stream) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  ht_status st = check_desc(A, "A");
  if (st) return st;
  st = check_desc(C, "C");
  if (st) return st;
  st = check_desc(S, "S");
  if (st) return st;
  if (A->d != C->d || A->d != S->d) return fail(HT_ESHAPE, "d differs");
  const int d = A->d;
  Tree tr(d);
  for (int mu = 0; mu < d; ++mu)
    if (A->n[mu] != C->n[mu] || A->n[mu] != S->n[mu]) return fail(HT_ESHAPE, "n differs");
  for (int t = 1; t < tr.nn; ++t)
    if (S->rank[t] != A->rank[t] + C->rank[t]) return fail(HT_ESHAPE, "S ranks must be rank_A + rank_C");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(HT_EINVAL, "alpha and beta must be finite");
  const long long s = std::max<long long>(A->log2_scale, C->log2_scale);
  const double a = std::ldexp(alpha, (int)std::max<long long>(-2000, A->log2_scale - s));
  const double c = std::ldexp(beta, (int)std::max<long long>(-2000, C->log2_scale - s));
  HT_HIP(hipSetDevice(ctx->device));
  Plan P;
  for (int mu = 0; mu < d; ++mu) {
    const int t = tr.leaf_node[mu];
    const int64_t n = A->n[mu];
    const int ka = A->rank[t], kc = C->rank[t];
    add_copy(P, A->leaf[mu], A->frame_dtype, S->leaf[mu], S->frame_dtype, ka, n, A->leaf_ld[mu], 1,
             S->leaf_ld[mu], 1, 1.0);
    add_copy(P, C->leaf[mu], C->frame_dtype, (char*)S->leaf[mu] + (size_t)ka * S->leaf_ld[mu] * esize(S->frame_dtype),
             S->frame_dtype, kc, n, C->leaf_ld[mu], 1, S->leaf_ld[mu], 1, 1.0);
  }
  for (int t = 0; t < tr.nn; ++t) {
    if (tr.is_leaf(t)) continue;
    const int s1 = tr.son1[t], s2 = tr.son2[t];
    const int K1 = S->rank[s1], K2 = S->rank[s2], Kt = t == 0 ? 1 : S->rank[t];
    const int sdt = t == 0 ? HT_F64 : S->transfer_dtype;
    const int adt = t == 0 ? HT_F64 : A->transfer_dtype, cdt = t == 0 ? HT_F64 : C->transfer_dtype;
    add_fill(P, S->transfer[t], (size_t)Kt * K1 * K2 * esize(sdt));
    const int at = t == 0 ? 1 : A->rank[t], a1 = A->rank[s1], a2 = A->rank[s2];
    const int ct = t == 0 ? 1 : C->rank[t], c1 = C->rank[s1], c2 = C->rank[s2];
    add_copy3(P, A->transfer[t], adt, S->transfer[t], sdt, at, a1, a2, (int64_t)a1 * a2, a2, 1, (int64_t)K1 * K2, K2, 1,
              t == 0 ? a : 1.0);
    const size_t off = t == 0 ? (size_t)a1 * K2 + a2 : ((size_t)at * K1 * K2 + (size_t)a1 * K2 + a2);
    add_copy3(P, C->transfer[t], cdt, (char*)S->transfer[t] + off * esize(sdt), sdt, ct, c1, c2, (int64_t)c1 * c2, c2, 1,
              (int64_t)K1 * K2, K2, 1, t == 0 ? c : 1.0);
  }
  if (out_log2_scale) *out_log2_scale = s;
  return run_plan(ctx, P, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"

// ================================================================== profiling
extern "C" {

ht_status ht_profile_enable(ht_context* ctx, int32_t on) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->prof = on != 0;
  return HT_OK;
}

ht_status ht_profile_read(ht_context* ctx, int32_t max_entries, ht_profile_entry* out, int32_t* n_out) {
  if (!ctx || !n_out) return fail(HT_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);   // launches append to the same lists
  for (auto& p : ctx->pending) {
    HT_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    HT_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    ProfAgg* a = nullptr;
    for (auto& x : ctx->agg)
      if (x.label == p.label && x.kernel == p.kernel) { a = &x; break; }
    if (!a) {
      ctx->agg.push_back(ProfAgg());
      a = &ctx->agg.back();
      a->label = p.label;
      a->kernel = p.kernel;
    }
    a->n += 1; a->ms += ms; a->flops += p.flops; a->bytes += p.bytes;
    ctx->free_events.push_back(p.a);
    ctx->free_events.push_back(p.b);
  }
  ctx->pending.clear();
  const int n = (int)ctx->agg.size();
  *n_out = n;
  for (int i = 0; i < n && i < max_entries && out; ++i) {
    std::memset(&out[i], 0, sizeof(ht_profile_entry));
    std::strncpy(out[i].label, ctx->agg[i].label.c_str(), sizeof(out[i].label) - 1);
    std::strncpy(out[i].kernel, ctx->agg[i].kernel.c_str(), sizeof(out[i].kernel) - 1);
    out[i].launches = ctx->agg[i].n;
    out[i].ms = ctx->agg[i].ms;
    out[i].flops = ctx->agg[i].flops;
    out[i].bytes = ctx->agg[i].bytes;
  }
  return HT_OK;
}

ht_status ht_profile_reset(ht_context* ctx) {
  if (!ctx) return fail(HT_EINVAL, "ctx is NULL");
  int32_t n = 0;
  ht_status s = ht_profile_read(ctx, 0, nullptr, &n);
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->agg.clear();
  return s;
}

}  // extern "C"

// ================================================================== bounds validation (host only)
// Builds a plan against fake, disjoint address ranges sized from the shapes
// (user buffers and every workspace allocation) and checks that every byte a
// kernel of the plan may touch lies inside one of them.
namespace {

struct FakeSpace {
  uintptr_t next = (uintptr_t)1 << 40;
  void* get(size_t bytes, const std::string& what) {
    next = (next + 4095) & ~(uintptr_t)4095;
    void* p = reinterpret_cast<void*>(next);
    reg(p, bytes, what);
    next += bytes + 4096;  // a gap: an overrun never lands in the neighbour
    return p;
  }
};

struct FakeTensor {
  std::vector<int64_t> n, ld;
  std::vector<int32_t> rank;
  std::vector<void*> leaf, transfer;
  ht_desc desc;
};

void fake_tensor(FakeSpace& F, const ht_desc* X, const std::vector<int>& ranks, int fdt, int tdt, FakeTensor& T,
                 const std::string& name) {
  const int d = X->d;
  Tree tr(d);
  T.n.assign(X->n, X->n + d);
  T.ld = T.n;
  T.rank.assign(ranks.begin(), ranks.end());
  T.leaf.assign(d, nullptr);
  T.transfer.assign(tr.nn, nullptr);
  for (int mu = 0; mu < d; ++mu)
    T.leaf[mu] = F.get((size_t)T.n[mu] * ranks[tr.leaf_node[mu]] * esize(fdt), name + " leaf");
  for (int t = 0; t < tr.nn; ++t) {
    if (tr.is_leaf(t)) continue;
    const int kt = t == 0 ? 1 : ranks[t];
    T.transfer[t] = F.get((size_t)kt * ranks[tr.son1[t]] * ranks[tr.son2[t]] * esize(t == 0 ? F64 : tdt),
                          name + " transfer");
  }
  T.desc = *X;
  T.desc.n = T.n.data();
  T.desc.rank = T.rank.data();
  T.desc.frame_dtype = fdt;
  T.desc.transfer_dtype = tdt;
  T.desc.leaf = T.leaf.data();
  T.desc.leaf_ld = T.ld.data();
  T.desc.transfer = T.transfer.data();
}

// [lo, hi) lies inside one registered region: with the regions sorted by
// start, some region that starts at or before lo must reach hi, i.e. the
// largest end among them is >= hi (regions may nest, as the zero-filled
// block around the accumulation targets does).
struct RegionIndex {
  const std::vector<Region>* src = nullptr;
  size_t n = 0;
  std::vector<uintptr_t> start, maxend;
};
static thread_local RegionIndex g_rindex;

bool inside(uintptr_t lo, uintptr_t hi) {
  RegionIndex& ix = g_rindex;
  if (ix.src != g_regions || ix.n != g_regions->size()) {
    std::vector<Region> v(*g_regions);
    std::sort(v.begin(), v.end(), [](const Region& a, const Region& b) { return a.lo < b.lo; });
    ix.start.resize(v.size());
    ix.maxend.resize(v.size());
    uintptr_t m = 0;
    for (size_t i = 0; i < v.size(); ++i) {
      ix.start[i] = v[i].lo;
      m = std::max<uintptr_t>(m, v[i].lo + v[i].bytes);
      ix.maxend[i] = m;
    }
    ix.src = g_regions;
    ix.n = g_regions->size();
  }
  const size_t i = std::upper_bound(ix.start.begin(), ix.start.end(), lo) - ix.start.begin();
  return i > 0 && ix.maxend[i - 1] >= hi;
}

ht_status check_range(const void* base, int64_t lo_el, int64_t hi_el, int esz, const std::string& what) {
  if (!base) return fail(HT_EINVAL, "validator: NULL pointer in " + what);
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  const uintptr_t lo = b + (uintptr_t)(lo_el * esz), hi = b + (uintptr_t)((hi_el + 1) * esz);
  if (!inside(lo, hi)) return fail(HT_EINVAL, "validator: out-of-bounds access in " + what);
  return HT_OK;
}

ht_status validate_plan(const Plan& P, int64_t m_entries) {
  g_rindex = RegionIndex();   // the regions are complete now: index them afresh
  auto at = [&](size_t off) { return P.table.data() + off; };
  int opi = 0;
  bool forked = false;   // second-stream launches only between a fork and its join
  for (const auto& op : P.ops) {
    if (op.kind == OP_FORK || op.kind == OP_JOIN) {
      // a fork may follow a fork (the second stream waits again); a join
      // closes them all
      if (op.kind == OP_JOIN && !forked) return fail(HT_EINVAL, "validator: join without a fork");
      forked = op.kind == OP_FORK;
      ++opi;
      continue;
    }
    if (op.stream && !forked) return fail(HT_EINVAL, "validator: second-stream launch outside a fork");
    const std::string tag = "op " + std::to_string(opi++) + " kind " + std::to_string(op.kind);
    ht_status s = HT_OK;
    if (op.kind == OP_GEMM) {
      const GemmDesc* ds = reinterpret_cast<const GemmDesc*>(at(op.toff));
      for (int i = 0; i < op.count; ++i) {
        const GemmDesc& g = ds[i];
        if (g.M <= 0 || g.N <= 0) continue;
        const int ea = esize(op.g.tA), eb = esize(op.g.tB), ec = esize(op.g.tC);
        const int nseg = g.nseg > 0 ? g.nseg : g.KB;
        const std::string w = tag + " desc " + std::to_string(i);
        if (g.nbatch > op.g.maxbatch) return fail(HT_EINVAL, "validator: batch " + w);
        const int tl = op.g.big ? 128 : 64;
        if (((g.M + tl - 1) / tl) * ((g.N + tl - 1) / tl) > op.g.maxtiles) return fail(HT_EINVAL, "validator: tiles " + w);
        if (op.g.sb) {   // the streamed kernel holds the whole reduction and the small side in LDS
          int kt = 0;
          for (int sg = 0; sg < nseg; ++sg) kt += g.nseg > 0 ? g.segK[sg] : g.K;
          const int rows = op.g.sb_swap ? g.N : g.M;
          if (g.KB != 1 || kt < 1 || kt > 128 || rows > 128 || (!op.g.sb_ring && rows > op.g.sb_rows))
            return fail(HT_EINVAL, "validator: streamed GEMM shape " + w);
        }
        if (g.msplit > 0) {   // two frames side by side: split-K Gram launches only
          if (!op.g.rk || op.g.rk_sym != 1 || g.kr || g.nseg > 0 || g.nbatch != 1 || g.msplit >= g.M || g.A != g.B)
            return fail(HT_EINVAL, "validator: split rows outside a Gram launch " + w);
          for (int sg = 0; sg < g.KB; ++sg) {
            const int64_t k0 = (int64_t)sg * g.sAkb, kl = (int64_t)(g.K - 1) * g.sAk;
            s = check_range(g.A, k0, k0 + (int64_t)(g.msplit - 1) * g.sAm + kl, ea, w + " A rows below the split");
            if (!s)
              s = check_range(g.A, k0 + (int64_t)g.msplit * g.sAm + g.a2off,
                              k0 + (int64_t)(g.M - 1) * g.sAm + g.a2off + kl, ea, w + " A rows from the split");
            if (s) return s;
          }
          s = check_range(g.C, 0, (int64_t)(g.M - 1) * g.sCm + (int64_t)(g.N - 1) * g.sCn, ec, w + " C");
          if (s) return s;
          continue;
        }
        for (int sg = 0; sg < nseg; ++sg) {
          const int ks = g.nseg > 0 ? g.segK[sg] : g.K;
          if (ks <= 0) continue;
          const int64_t bat = (int64_t)(g.nbatch - 1);
          if (g.kr) {
            s = check_range(g.krY1, 0, (int64_t)(g.M - 1) * g.krld1 + (ks - 1) / g.krK2, 8, w + " KR1");
            if (!s) s = check_range(g.krY2, 0, (int64_t)(g.M - 1) * g.krld2 + std::min(ks, g.krK2) - 1, 8, w + " KR2");
          } else {
            const void* Ab = g.nseg > 0 ? g.segA[sg] : g.A;
            const int64_t a0 = g.nseg > 0 ? 0 : (int64_t)sg * g.sAkb;
            const int64_t sak = g.nseg > 0 ? g.segAk[sg] : g.sAk;
            s = check_range(Ab, a0, a0 + (int64_t)(g.M - 1) * g.sAm + (int64_t)(ks - 1) * sak + bat * g.sAb, ea, w + " A");
          }
          if (s) return s;
          const int64_t b0 = g.nseg > 0 ? g.segBoff[sg] : (int64_t)sg * g.sBkb;
          s = check_range(g.B, b0, b0 + (int64_t)(ks - 1) * g.sBk + (int64_t)(g.N - 1) * g.sBn + bat * g.sBb, eb,
                          w + " B");
          if (s) return s;
        }
        s = check_range(g.C, 0, (int64_t)(g.M - 1) * g.sCm + (int64_t)(g.N - 1) * g.sCn + (int64_t)(g.nbatch - 1) * g.sCb,
                        ec, w + " C");
        if (s) return s;
        if (g.alpha_dev) { s = check_range(g.alpha_dev, 0, 0, 8, w + " alpha"); if (s) return s; }
      }
    } else if (op.kind == OP_CHOL1 || op.kind == OP_CHOL2 || op.kind == OP_EIG || op.kind == OP_RANK ||
               op.kind == OP_PROJPREP || op.kind == OP_SIGMA) {
      const SmallArgs* as = reinterpret_cast<const SmallArgs*>(at(op.toff));
      for (int i = 0; i < op.count; ++i) {
        const SmallArgs& a = as[i];
        const int64_t kk = (int64_t)a.K * a.K;
        const std::string w = tag + " node " + std::to_string(a.node);
        if (a.K < 1 || a.K > KMAX) return fail(HT_EINVAL, "validator: K " + w);
        auto chk = [&](const void* p, int64_t n, int e, const char* nm) -> ht_status {
          return check_range(p, 0, n - 1, e, w + " " + nm);
        };
        if (op.kind == OP_CHOL1 || op.kind == OP_CHOL2) {
          if ((s = chk(a.G, kk, 8, "G")) || (s = chk(a.G2, kk, 8, "G2")) || (s = chk(a.R1, kk, 8, "R1")) ||
              (s = chk(a.Ri1, kk, 8, "Ri1")))
            return s;
          if (op.kind == OP_CHOL2 && ((s = chk(a.R, kk, 8, "R")) || (s = chk(a.Ri, kk, 8, "Ri")) ||
                                      (s = chk(a.Rf, kk, esize(a.rf_type), "Rf"))))
            return s;
        } else if (op.kind == OP_EIG) {
          if ((s = chk(a.Bh, kk, 8, "Bh")) || (s = chk(a.Q, kk, 8, "Q")) || (s = chk(a.lam, a.K, 8, "lam")) ||
              (s = chk(a.scratch, eig_scratch_doubles(a.K), 8, "scratch")))
            return s;
        } else if (op.kind == OP_RANK) {
          if ((s = chk(a.lam, a.K, 8, "lam")) || (s = chk(a.rank_dev, 1, 4, "rank"))) return s;
        } else if (op.kind == OP_PROJPREP) {
          if ((s = chk(a.Q, kk, 8, "Q")) || (s = chk(a.rank_dev, 1, 4, "rank")) || (s = chk(a.lam, a.K, 8, "lam")))
            return s;
          if (a.Qm && (s = chk(a.Qm, (int64_t)a.K * a.rcap, 8, "Qm"))) return s;
          if (a.QmT && (s = chk(a.QmT, (int64_t)a.K * a.rcap, esize(a.rf_type), "QmT"))) return s;
          if (a.sigma_out && (s = chk(a.sigma_out, KMAX, 8, "sigma"))) return s;
          if (a.rcap < 1 || a.rcap > a.K) return fail(HT_EINVAL, "validator: rcap " + w);
        } else if (op.kind == OP_SIGMA) {
          if ((s = chk(a.lam, a.K, 8, "lam"))) return s;
        }
      }
    } else if (op.kind == OP_FILL) {
      const FillRec* fr = reinterpret_cast<const FillRec*>(at(op.toff));
      for (int i = 0; i < op.count; ++i) {
        if (fr[i].bytes > op.bytes || (fr[i].bytes & 3)) return fail(HT_EINVAL, "validator: fill size " + tag);
        if (fr[i].bytes && (s = check_range(fr[i].p, 0, (int64_t)fr[i].bytes / 4 - 1, 4, tag + " fill"))) return s;
      }
    } else if (op.kind == OP_COPY) {
      const CopyRec* cr = reinterpret_cast<const CopyRec*>(at(op.toff));
      for (int i = 0; i < op.count; ++i) {
        const CopyRec& c = cr[i];
        const int64_t n0 = c.n0, n1 = c.n1, n2 = c.n2;
        if (n0 * n1 * n2 > op.c[0]) return fail(HT_EINVAL, "validator: copy size " + tag);
        if (n0 * n1 * n2 == 0) continue;
        if ((s = check_range(c.src, 0, (n0 - 1) * c.s0 + (n1 - 1) * c.s1 + (n2 - 1) * c.s2, esize(c.tsrc),
                             tag + " copy src")))
          return s;
        if ((s = check_range(c.dst, 0, (n0 - 1) * c.d0 + (n1 - 1) * c.d1 + (n2 - 1) * c.d2, esize(c.tdst),
                             tag + " copy dst")))
          return s;
      }
    } else if (op.kind == OP_SETSTATE || op.kind == OP_WRITESCALE || op.kind == OP_ROOTNORM) {
      const StateRec* sr = reinterpret_cast<const StateRec*>(at(op.toff));
      for (int i = 0; i < op.count; ++i) {
        const StateRec& r = sr[i];
        if ((s = check_range(r.st, 0, 0, sizeof(GlobalState), tag + " state"))) return s;
        if (op.kind == OP_ROOTNORM && (s = check_range(r.BD, 0, (int64_t)r.K1 * r.K2 - 1, 8, tag + " root")))
          return s;
        if (op.kind == OP_WRITESCALE) {
          if (r.out_scale && (s = check_range(r.out_scale, 0, 0, 8, tag + " scale"))) return s;
          if (r.flags && (s = check_range(r.flags, 0, 0, 4, tag + " flags"))) return s;
          if (r.root_rank && (s = check_range(r.root_rank, 0, 0, 4, tag + " ranks"))) return s;
        }
      }
    } else if (op.kind == OP_EGATHER || op.kind == OP_ENORM) {
      const EntryNode* en = reinterpret_cast<const EntryNode*>(at(op.toff));
      const int64_t mc = op.c[0];
      for (int i = 0; i < op.count; ++i) {
        const std::string w = tag + " entry node " + std::to_string(i);
        if ((s = check_range(en[i].rows, 0, mc * en[i].k - 1, 8, w + " rows")) ||
            (s = check_range(en[i].expo, 0, mc - 1, 4, w + " expo")))
          return s;
        if (op.kind == OP_EGATHER) {
          if ((s = check_range(op.p0, 0, mc * op.i0 - 1, 4, w + " idx"))) return s;
        }
        if (en[i].expo1 && (s = check_range(en[i].expo1, 0, mc - 1, 4, w + " expo1"))) return s;
        if (en[i].expo2 && (s = check_range(en[i].expo2, 0, mc - 1, 4, w + " expo2"))) return s;
      }
    } else if (op.kind == OP_KRON) {
      const KronRec* kr = reinterpret_cast<const KronRec*>(at(op.toff));
      for (int i = 0; i < op.count; ++i) {
        const KronRec& r = kr[i];
        const std::string w = tag + " kron record " + std::to_string(i);
        const int64_t nh = (int64_t)r.P * r.Q * r.R, nb = (int64_t)r.I * r.J * r.L;
        if (nh < 1 || nb < 1 || nh * nb > op.c[0] || (int64_t)r.P * r.I > op.c[1])
          return fail(HT_EINVAL, "validator: kron size " + w);
        if ((s = check_range(r.H, 0, nh - 1, esize(r.tH), w + " H")) ||
            (s = check_range(r.B, 0, nb - 1, esize(r.tB), w + " B")) ||
            (s = check_range(r.F, 0, nh * nb - 1, esize(r.tF), w + " F")))
          return s;
      }
    } else if (op.kind == OP_PHI) {
      const PhiRec* pr = reinterpret_cast<const PhiRec*>(at(op.toff));
      for (int i = 0; i < op.count; ++i) {
        const PhiRec& r = pr[i];
        const std::string w = tag + " phi record " + std::to_string(i);
        if (r.n < 1 || (r.mode == 1 && r.n != 1)) return fail(HT_EINVAL, "validator: phi size " + w);
        if ((s = check_range(r.P, 0, r.n - 1, 8, w + " P"))) return s;
        if (r.E && (s = check_range(r.E, 0, 0, 8, w + " E"))) return s;
        if (r.E1 && (s = check_range(r.E1, 0, 0, 8, w + " E1"))) return s;
        if (r.E2 && (s = check_range(r.E2, 0, 0, 8, w + " E2"))) return s;
        if (r.add_dev && (s = check_range(r.add_dev, 0, 0, 8, w + " add"))) return s;
        if (r.flags && (s = check_range(r.flags, 0, 0, 4, w + " flags"))) return s;
        if (r.mode >= 1 && ((s = check_range(r.out_val, 0, 0, 8, w + " out")) ||
                            (s = check_range(r.out_log2, 0, 0, 8, w + " out_log2"))))
          return s;
      }
    } else if (op.kind == OP_EFINISH) {
      if ((s = check_range(op.p0, 0, op.c[0] - 1, 8, tag + " vals")) || (s = check_range(op.p1, 0, op.c[0] - 1, 4, tag + " expo")) ||
          (s = check_range(op.p2, 0, op.c[0] - 1, 8, tag + " out")))
        return s;
    }
    if (op.kind == OP_RANK) {   // each tensor's node range lies inside the launch's arguments
      const StateRec* sr = reinterpret_cast<const StateRec*>(at(op.toff2));
      for (int i = 0; i < op.count2; ++i) {
        if (sr[i].a0 < 0 || sr[i].na < 1 || sr[i].a0 + sr[i].na > op.count)
          return fail(HT_EINVAL, "validator: rank range " + tag);
        if ((s = check_range(sr[i].st, 0, 0, sizeof(GlobalState), tag + " state"))) return s;
      }
    }
  }
  if (forked) return fail(HT_EINVAL, "validator: plan ends with the second stream not joined");
  (void)m_entries;
  return HT_OK;
}

struct RegionScope {
  std::vector<Region> regions;
  RegionScope() { g_regions = &regions; g_rindex = RegionIndex(); }
  ~RegionScope() { g_regions = nullptr; g_rindex = RegionIndex(); }
};

}  // namespace

extern "C" {

ht_status ht_debug_validate_truncate(const ht_desc* X, int32_t n_in, const ht_trunc_opts* opts) {
  RegionScope scope;
  size_t need = 0;
  ht_status st = ht_truncate_workspace(nullptr, X, n_in, opts, &need);
  if (st) return st;
  FakeSpace F;
  std::vector<FakeTensor> fx(n_in);
  std::vector<ht_desc> xs(n_in);
  const int d = X[0].d;
  Tree tr(d);
  for (int c = 0; c < n_in; ++c) {
    std::vector<int> rk(X[c].rank, X[c].rank + tr.nn);
    fake_tensor(F, &X[c], rk, X[c].frame_dtype, X[c].transfer_dtype, fx[c], "X");
    xs[c] = fx[c].desc;
  }
  SumInfo S;
  if ((st = sum_info(xs.data(), nullptr, n_in, S))) return st;
  std::vector<int> rc(tr.nn, 1);
  for (int t = 1; t < tr.nn; ++t)
    rc[t] = opts->mode == HT_RANK_FIXED ? std::min(opts->ranks[t], S.K[t])
                                        : (opts->max_rank > 0 ? std::min(opts->max_rank, S.K[t]) : S.K[t]);
  if (opts->mode == HT_RANK_TOL) rc[tr.son1[0]] = rc[tr.son2[0]] = std::min(rc[tr.son1[0]], rc[tr.son2[0]]);
  FakeTensor fo;
  const int T = opts->precision == HT_PREC_MIXED ? HT_F32 : HT_F64;
  fake_tensor(F, &X[0], rc, T, T, fo, "out");
  void* ranks = F.get((size_t)tr.nn * 4, "out_ranks");
  void* scale = F.get(8, "out_scale");
  void* flags = F.get(4, "flags");
  void* sigma = F.get((size_t)tr.nn * KMAX * 8, "sigma");
  void* ws = F.get(need, "ws-total");
  g_regions->pop_back();  // only the individual workspace allocations count
  Plan P;
  std::vector<double> coef(n_in, 1.0);
  st = build_truncate(nullptr, xs.data(), coef.data(), n_in, opts, &fo.desc, (int32_t*)ranks, (int64_t*)scale,
                      (uint32_t*)flags, (double*)sigma, ws, P, nullptr);
  if (st) return st;
  return validate_plan(P, 0);
}

ht_status ht_debug_plan_key_repeats(const ht_desc* X, int32_t n_in, const ht_trunc_opts* opts, int32_t* equal,
                                    uint64_t* hash) {
  if (!X || !opts || !equal || n_in < 1 || n_in > MAX_SEG) return fail(HT_EINVAL, "bad argument");
  RegionScope scope;
  size_t need = 0;
  ht_status st = ht_truncate_workspace(nullptr, X, n_in, opts, &need);
  if (st) return st;
  FakeSpace F;
  std::vector<FakeTensor> fx(n_in);
  std::vector<ht_desc> xs(n_in);
  Tree tr(X[0].d);
  for (int c = 0; c < n_in; ++c) {
    std::vector<int> rk(X[c].rank, X[c].rank + tr.nn);
    fake_tensor(F, &X[c], rk, X[c].frame_dtype, X[c].transfer_dtype, fx[c], "X");
    xs[c] = fx[c].desc;
  }
  SumInfo S;
  if ((st = sum_info(xs.data(), nullptr, n_in, S))) return st;
  std::vector<int> rc(tr.nn, 1);
  for (int t = 1; t < tr.nn; ++t)
    rc[t] = opts->mode == HT_RANK_FIXED ? std::min(opts->ranks[t], S.K[t])
                                        : (opts->max_rank > 0 ? std::min(opts->max_rank, S.K[t]) : S.K[t]);
  if (opts->mode == HT_RANK_TOL) rc[tr.son1[0]] = rc[tr.son2[0]] = std::min(rc[tr.son1[0]], rc[tr.son2[0]]);
  FakeTensor fo;
  const int T = opts->precision == HT_PREC_MIXED ? HT_F32 : HT_F64;
  fake_tensor(F, &X[0], rc, T, T, fo, "out");
  void* scale = F.get(8, "out_scale");
  void* ws = F.get(need, "ws-total");
  std::vector<double> coef(n_in, 1.0);
  std::vector<unsigned char> keys[2];
  for (int rep = 0; rep < 2; ++rep) {
    Plan P;
    st = build_truncate(nullptr, xs.data(), coef.data(), n_in, opts, &fo.desc, nullptr, (int64_t*)scale, nullptr,
                        nullptr, ws, P, nullptr);
    if (st) return st;
    build_key(P);
    keys[rep].swap(P.key);
  }
  *equal = keys[0] == keys[1] ? 1 : 0;
  if (hash) {   // FNV-1a of the first key
    uint64_t h = 1469598103934665603ull;
    for (unsigned char b : keys[0]) h = (h ^ b) * 1099511628211ull;
    *hash = h;
  }
  return HT_OK;
}

ht_status ht_debug_validate_truncate_batched(int32_t count, const ht_desc* X, const int32_t* n_in,
                                             const ht_trunc_opts* opts, int32_t* n_launches) {
  RegionScope scope;
  size_t need = 0;
  ht_status st = ht_truncate_batched_workspace(nullptr, count, X, n_in, opts, &need);
  if (st) return st;
  FakeSpace F;
  int64_t tot = 0;
  for (int c = 0; c < count; ++c) tot += n_in[c];
  std::vector<FakeTensor> fx(tot), fo(count);
  std::vector<ht_desc> xs(tot), outs(count);
  std::vector<int32_t*> ranks(count);
  std::vector<double*> sigma(count);
  int64_t first = 0;
  for (int c = 0; c < count; ++c) {
    const int d = X[first].d;
    Tree tr(d);
    for (int i = 0; i < n_in[c]; ++i) {
      const ht_desc& Xi = X[first + i];
      std::vector<int> rk(Xi.rank, Xi.rank + tr.nn);
      fake_tensor(F, &Xi, rk, Xi.frame_dtype, Xi.transfer_dtype, fx[first + i], "X");
      xs[first + i] = fx[first + i].desc;
    }
    SumInfo S;
    if ((st = sum_info(xs.data() + first, nullptr, n_in[c], S))) return st;
    const ht_trunc_opts& o = opts[c];
    std::vector<int> rc(tr.nn, 1);
    for (int t = 1; t < tr.nn; ++t)
      rc[t] = o.mode == HT_RANK_FIXED ? std::min(o.ranks[t], S.K[t])
                                      : (o.max_rank > 0 ? std::min(o.max_rank, S.K[t]) : S.K[t]);
    if (o.mode == HT_RANK_TOL) rc[tr.son1[0]] = rc[tr.son2[0]] = std::min(rc[tr.son1[0]], rc[tr.son2[0]]);
    const int T = o.precision == HT_PREC_MIXED ? HT_F32 : HT_F64;
    fake_tensor(F, &X[first], rc, T, T, fo[c], "out");
    outs[c] = fo[c].desc;
    ranks[c] = (int32_t*)F.get((size_t)tr.nn * 4, "out_ranks");
    sigma[c] = (double*)F.get((size_t)tr.nn * KMAX * 8, "sigma");
    first += n_in[c];
  }
  void* scale = F.get((size_t)count * 8, "out_scale");
  void* flags = F.get((size_t)count * 4, "flags");
  // the workspace: one region per problem, as the library lays it out
  std::vector<size_t> part(count);
  first = 0;
  for (int c = 0; c < count; ++c) {
    if ((st = ht_truncate_workspace(nullptr, xs.data() + first, n_in[c], &opts[c], &part[c]))) return st;
    part[c] = align256(part[c]);
    first += n_in[c];
  }
  void* ws = F.get(need, "ws-total");
  g_regions->pop_back();
  size_t acc = 0;
  for (int c = 0; c < count; ++c) acc += part[c];
  if (acc != need) return fail(HT_EINVAL, "validator: batched workspace size differs from the sum of its parts");
  Plan M;
  std::vector<double> coef(tot, 1.0);
  st = build_truncate_batched(nullptr, count, xs.data(), n_in, coef.data(), opts, outs.data(), ranks.data(),
                              (int64_t*)scale, (uint32_t*)flags, sigma.data(), ws, M, nullptr);
  if (st) return st;
  if (n_launches) *n_launches = (int32_t)M.ops.size();
  return validate_plan(M, 0);
}

ht_status ht_debug_validate_orthogonalize(const ht_desc* X, int32_t precision) {
  RegionScope scope;
  size_t need = 0;
  ht_status st = ht_orthogonalize_workspace(nullptr, X, precision, &need);
  if (st) return st;
  FakeSpace F;
  Tree tr(X->d);
  FakeTensor fx;
  std::vector<int> rk(X->rank, X->rank + tr.nn);
  fake_tensor(F, X, rk, X->frame_dtype, X->transfer_dtype, fx, "X");
  void* scale = F.get(8, "scale");
  void* ws = F.get(need, "ws-total");
  g_regions->pop_back();
  Plan P;
  st = build_orth(&fx.desc, precision, (int64_t*)scale, nullptr, ws, P, nullptr);
  if (st) return st;
  return validate_plan(P, 0);
}

ht_status ht_debug_validate_inner(const ht_desc* X, const ht_desc* Y) {
  RegionScope scope;
  size_t need = 0;
  ht_status st = ht_inner_workspace(nullptr, X, Y, &need);
  if (st) return st;
  FakeSpace F;
  Tree tr(X->d);
  FakeTensor fx, fy;
  std::vector<int> rx(X->rank, X->rank + tr.nn), ry(Y->rank, Y->rank + tr.nn);
  fake_tensor(F, X, rx, X->frame_dtype, X->transfer_dtype, fx, "X");
  fake_tensor(F, Y, ry, Y->frame_dtype, Y->transfer_dtype, fy, "Y");
  void* val = F.get(8, "out_val");
  void* lg = F.get(8, "out_log2");
  void* flags = F.get(4, "flags");
  void* ws = F.get(need, "ws-total");
  g_regions->pop_back();
  Plan P;
  st = build_inner(&fx.desc, &fy.desc, (double*)val, (int64_t*)lg, (uint32_t*)flags, ws, P, nullptr);
  if (st) return st;
  return validate_plan(P, 0);
}

ht_status ht_debug_validate_norm(const ht_desc* X, int32_t n_in) {
  RegionScope scope;
  size_t need = 0;
  ht_status st = ht_norm_workspace(nullptr, X, n_in, &need);
  if (st) return st;
  FakeSpace F;
  Tree tr(X[0].d);
  std::vector<FakeTensor> fx(n_in);
  std::vector<ht_desc> xs(n_in);
  for (int c = 0; c < n_in; ++c) {
    std::vector<int> rk(X[c].rank, X[c].rank + tr.nn);
    fake_tensor(F, &X[c], rk, X[c].frame_dtype, X[c].transfer_dtype, fx[c], "X");
    xs[c] = fx[c].desc;
  }
  void* val = F.get(8, "out_val");
  void* lg = F.get(8, "out_log2");
  void* flags = F.get(4, "flags");
  void* ws = F.get(need, "ws-total");
  g_regions->pop_back();
  Plan P;
  std::vector<double> coef(n_in, 1.0);
  st = build_norm(xs.data(), coef.data(), n_in, (double*)val, (int64_t*)lg, (uint32_t*)flags, ws, P, nullptr);
  if (st) return st;
  return validate_plan(P, 0);
}

ht_status ht_debug_validate_apply(const ht_desc* L, const ht_desc* A) {
  RegionScope scope;
  FakeSpace F;
  Tree tr(A->d);
  FakeTensor fl, fa, fc;
  std::vector<int> rl(L->rank, L->rank + tr.nn), ra(A->rank, A->rank + tr.nn), rc(tr.nn, 1);
  for (int t = 1; t < tr.nn; ++t) rc[t] = rl[t] * ra[t];
  fake_tensor(F, L, rl, L->frame_dtype, L->transfer_dtype, fl, "L");
  fake_tensor(F, A, ra, A->frame_dtype, A->transfer_dtype, fa, "A");
  fake_tensor(F, A, rc, A->frame_dtype, A->transfer_dtype, fc, "C");
  Plan P;
  ht_status st = build_apply(&fl.desc, &fa.desc, &fc.desc, P);
  if (st) return st;
  return validate_plan(P, 0);
}

ht_status ht_debug_validate_gramians(const ht_desc* X) {
  RegionScope scope;
  size_t need = 0;
  ht_status st = ht_gramians_workspace(nullptr, X, &need);
  if (st) return st;
  FakeSpace F;
  Tree tr(X->d);
  FakeTensor fx;
  std::vector<int> rk(X->rank, X->rank + tr.nn);
  fake_tensor(F, X, rk, X->frame_dtype, X->transfer_dtype, fx, "X");
  std::vector<double*> bh(tr.nn, nullptr), sg(tr.nn, nullptr);
  for (int t = 1; t < tr.nn; ++t) {
    bh[t] = (double*)F.get((size_t)rk[t] * rk[t] * 8, "bhat");
    sg[t] = (double*)F.get((size_t)rk[t] * 8, "sigma");
  }
  void* units = F.get(8, "units");
  void* ws = F.get(need, "ws-total");
  g_regions->pop_back();
  Plan P;
  st = build_gram(&fx.desc, bh.data(), sg.data(), (int64_t*)units, ws, P, nullptr);
  if (st) return st;
  return validate_plan(P, 0);
}

ht_status ht_debug_validate_entries(const ht_desc* X, int64_t m) {
  RegionScope scope;
  size_t need = 0;
  ht_status st = ht_entries_workspace(nullptr, X, m, &need);
  if (st) return st;
  FakeSpace F;
  Tree tr(X->d);
  FakeTensor fx;
  std::vector<int> rk(X->rank, X->rank + tr.nn);
  fake_tensor(F, X, rk, X->frame_dtype, X->transfer_dtype, fx, "X");
  void* idx = F.get((size_t)m * X->d * 4, "idx");
  void* out = F.get((size_t)m * 8, "out");
  void* ws = F.get(need, "ws-total");
  g_regions->pop_back();
  Plan P;
  st = build_entries(&fx.desc, m, (const int32_t*)idx, (double*)out, ws, P, nullptr);
  if (st) return st;
  return validate_plan(P, m);
}

}  // extern "C"
