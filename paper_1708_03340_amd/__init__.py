"""Python binding of libht.so, the MI355X hierarchical-SVD library for tensors in
the Hierarchical Tucker format (C ABI in include/ht.h).

The functions here only marshal arguments: torch tensors supply device memory
and the current HIP stream, every computation runs in the library's kernels.
Importing this package does not load the library; the first call does, and it
raises if libht.so has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libht.so")

HT_F64, HT_F32 = 0, 1
HT_PREC_FP64, HT_PREC_MIXED = 0, 1
HT_RANK_FIXED, HT_RANK_TOL = 0, 1
HT_FLAG_RANK_DEFICIENT, HT_FLAG_NONFINITE, HT_FLAG_CAPPED, HT_FLAG_NOCONV = 1, 2, 4, 8
KMAX = 128
NOALLOC_SCRATCH_BYTES = 64 << 20   # HT_NOALLOC_SCRATCH_BYTES

EXPORTS = [
    "ht_create_context", "ht_destroy_context", "ht_status_string", "ht_last_error", "ht_version",
    "ht_tree", "ht_add", "ht_orthogonalize_workspace", "ht_orthogonalize", "ht_gramians_workspace",
    "ht_gramians", "ht_truncate_workspace", "ht_truncate", "ht_truncate_batched_workspace",
    "ht_truncate_batched", "ht_entries_workspace", "ht_entries", "ht_truncate_noalloc",
    "ht_inner_workspace", "ht_inner", "ht_norm_workspace", "ht_norm", "ht_apply",
    "ht_profile_enable", "ht_profile_read", "ht_profile_reset",
]


class HtDesc(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("n", ctypes.POINTER(ctypes.c_int64)),
        ("rank", ctypes.POINTER(ctypes.c_int32)),
        ("frame_dtype", ctypes.c_int32),
        ("transfer_dtype", ctypes.c_int32),
        ("leaf", ctypes.POINTER(ctypes.c_void_p)),
        ("leaf_ld", ctypes.POINTER(ctypes.c_int64)),
        ("transfer", ctypes.POINTER(ctypes.c_void_p)),
        ("log2_scale", ctypes.c_int64),
    ]


class HtTruncOpts(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("ranks", ctypes.POINTER(ctypes.c_int32)),
        ("eps", ctypes.c_double),
        ("eps_relative", ctypes.c_int32),
        ("max_rank", ctypes.c_int32),
        ("precision", ctypes.c_int32),
    ]


class HtProfileEntry(ctypes.Structure):
    _fields_ = [
        ("label", ctypes.c_char * 48),
        ("kernel", ctypes.c_char * 48),
        ("launches", ctypes.c_int64),
        ("ms", ctypes.c_double),
        ("flops", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


class HTError(RuntimeError):
    pass


_LIB = None


def lib(path: Optional[str] = None):
    """Load libht.so (raises if it is missing)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise HTError(f"{p} is not built; run paper_1708_03340_amd.build.build()")
    L = ctypes.CDLL(p)
    P, I32, I64, VP = ctypes.POINTER, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.ht_status_string.restype = ctypes.c_char_p
    L.ht_last_error.restype = ctypes.c_char_p
    L.ht_version.restype = I32
    L.ht_create_context.argtypes = [ctypes.c_int, P(VP)]
    L.ht_destroy_context.argtypes = [VP]
    L.ht_destroy_context.restype = None
    L.ht_tree.argtypes = [I32] + [P(I32)] * 7
    L.ht_add.argtypes = [VP, ctypes.c_double, P(HtDesc), ctypes.c_double, P(HtDesc), P(HtDesc), P(I64), VP]
    L.ht_orthogonalize_workspace.argtypes = [VP, P(HtDesc), I32, P(ctypes.c_size_t)]
    L.ht_orthogonalize.argtypes = [VP, P(HtDesc), I32, VP, VP, VP, ctypes.c_size_t, VP]
    L.ht_gramians_workspace.argtypes = [VP, P(HtDesc), P(ctypes.c_size_t)]
    L.ht_gramians.argtypes = [VP, P(HtDesc), P(VP), P(VP), VP, VP, ctypes.c_size_t, VP]
    L.ht_truncate_workspace.argtypes = [VP, P(HtDesc), I32, P(HtTruncOpts), P(ctypes.c_size_t)]
    L.ht_truncate.argtypes = [VP, P(HtDesc), P(ctypes.c_double), I32, P(HtTruncOpts), P(HtDesc), VP, VP, VP,
                              VP, VP, ctypes.c_size_t, VP]
    L.ht_truncate_noalloc.argtypes = [VP, P(HtDesc), P(ctypes.c_double), I32, P(HtTruncOpts), P(HtDesc), VP,
                                      VP, VP, VP, VP]
    L.ht_inner_workspace.argtypes = [VP, P(HtDesc), P(HtDesc), P(ctypes.c_size_t)]
    L.ht_inner.argtypes = [VP, P(HtDesc), P(HtDesc), VP, VP, VP, VP, ctypes.c_size_t, VP]
    L.ht_norm_workspace.argtypes = [VP, P(HtDesc), I32, P(ctypes.c_size_t)]
    L.ht_norm.argtypes = [VP, P(HtDesc), P(ctypes.c_double), I32, VP, VP, VP, VP, ctypes.c_size_t, VP]
    L.ht_apply.argtypes = [VP, P(HtDesc), P(HtDesc), P(HtDesc), VP]
    L.ht_truncate_batched_workspace.argtypes = [VP, I32, P(HtDesc), P(I32), P(HtTruncOpts), P(ctypes.c_size_t)]
    L.ht_truncate_batched.argtypes = [VP, I32, P(HtDesc), P(I32), P(ctypes.c_double), P(HtTruncOpts), P(HtDesc),
                                      P(VP), VP, VP, P(VP), VP, ctypes.c_size_t, VP]
    L.ht_entries_workspace.argtypes = [VP, P(HtDesc), I64, P(ctypes.c_size_t)]
    L.ht_entries.argtypes = [VP, P(HtDesc), I64, VP, VP, VP, ctypes.c_size_t, VP]
    L.ht_profile_enable.argtypes = [VP, I32]
    L.ht_profile_read.argtypes = [VP, I32, P(HtProfileEntry), P(I32)]
    L.ht_profile_reset.argtypes = [VP]
    for name in EXPORTS:
        if name not in ("ht_status_string", "ht_last_error", "ht_version", "ht_destroy_context"):
            getattr(L, name).restype = ctypes.c_int
    if path is None:
        _LIB = L
    return L


def _check(status: int):
    if status != 0:
        L = lib()
        msg = L.ht_last_error().decode()
        raise HTError(f"{L.ht_status_string(status).decode()}: {msg}")


# ---------------------------------------------------------------- tree
def ht_tree(d: int):
    """Balanced tree of eq. (balanced) as numpy arrays (preorder)."""
    nn = 2 * d - 1
    arrs = [np.zeros(nn, dtype=np.int32) for _ in range(7)]
    ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for a in arrs]
    _check(lib().ht_tree(d, *ptrs))
    keys = ["parent", "son1", "son2", "lo", "hi", "depth", "height"]
    return dict(zip(keys, arrs))


# ---------------------------------------------------------------- context
class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().ht_create_context(device, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().ht_destroy_context(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_CTX = {}


def ht_create_context(device: int = 0) -> Context:
    if device not in _CTX:
        _CTX[device] = Context(device)
    return _CTX[device]


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dt(torch_dtype):
    import torch
    return HT_F32 if torch_dtype == torch.float32 else HT_F64


# ---------------------------------------------------------------- device-resident HT tensor
class DeviceHT:
    """An HT tensor in device memory (torch tensors).

    leaves[mu]:   tensor of shape (k_mu, n_mu) -- the column-major n_mu x k_mu frame;
    transfer[t]:  tensor of shape (k_t, k_s1, k_s2) for inner t (None at leaves),
                  (k_t1, k_t2) float64 for the root t = 0;
    log2_scale:   int, or a 1-element int64 device tensor written by the library.
    """

    def __init__(self, d, n, ranks, leaves, transfer, log2_scale=0):
        self.d = int(d)
        self.n = [int(x) for x in n]
        self.ranks = [int(r) for r in ranks]
        self.leaves = leaves
        self.transfer = transfer
        self.log2_scale = log2_scale
        self._keep = None

    # -- construction
    @staticmethod
    def empty(d, n, ranks, frame_dtype=None, transfer_dtype=None, device="cuda"):
        import torch
        frame_dtype = frame_dtype or torch.float64
        transfer_dtype = transfer_dtype or torch.float64
        tr = ht_tree(d)
        nn = 2 * d - 1
        ns = [int(n)] * d if np.isscalar(n) else list(n)
        leaves = [None] * d
        transfer = [None] * nn
        for t in range(nn):
            s1, s2 = int(tr["son1"][t]), int(tr["son2"][t])
            if s1 < 0:
                mu = int(tr["lo"][t])
                leaves[mu] = torch.zeros((ranks[t], ns[mu]), dtype=frame_dtype, device=device)
            elif t == 0:
                transfer[t] = torch.zeros((ranks[s1], ranks[s2]), dtype=torch.float64, device=device)
            else:
                transfer[t] = torch.zeros((ranks[t], ranks[s1], ranks[s2]), dtype=transfer_dtype, device=device)
        r = list(ranks)
        r[0] = 1
        return DeviceHT(d, ns, r, leaves, transfer, 0)

    @staticmethod
    def from_input(inp, device="cuda", frame_dtype=None, transfer_dtype=None):
        """From an htsynth.HTInput (inner[j] = j-th non-root inner node in preorder)."""
        import torch
        tr = ht_tree(inp.d)
        nn = 2 * inp.d - 1
        fdt = frame_dtype or (torch.float32 if inp.leaves[0].dtype == np.float32 else torch.float64)
        tdt = transfer_dtype or (torch.float32 if inp.inner and inp.inner[0].dtype == np.float32 else torch.float64)
        leaves = [torch.from_numpy(np.ascontiguousarray(u.T)).to(device=device, dtype=fdt) for u in inp.leaves]
        transfer = [None] * nn
        transfer[0] = torch.from_numpy(np.ascontiguousarray(inp.root, dtype=np.float64)).to(device)
        j = 0
        ranks = [1] * nn
        for t in range(nn):
            if int(tr["son1"][t]) < 0:
                ranks[t] = inp.leaves[int(tr["lo"][t])].shape[1]
            elif t != 0:
                transfer[t] = torch.from_numpy(np.ascontiguousarray(inp.inner[j])).to(device=device, dtype=tdt)
                ranks[t] = inp.inner[j].shape[0]
                j += 1
        return DeviceHT(inp.d, inp.n, ranks, leaves, transfer, inp.log2_scale)

    @staticmethod
    def from_arrays(d, U, B, log2_scale=0, device="cuda", frame_dtype=None, transfer_dtype=None):
        """From host arrays: U[mu] (n x k), B[t] per preorder node (None at leaves)."""
        import torch
        fdt = frame_dtype or torch.float64
        tdt = transfer_dtype or torch.float64
        nn = 2 * d - 1
        tr = ht_tree(d)
        leaves = [torch.from_numpy(np.ascontiguousarray(np.asarray(u).T)).to(device=device, dtype=fdt) for u in U]
        transfer = [None] * nn
        ranks = [1] * nn
        for t in range(nn):
            if int(tr["son1"][t]) < 0:
                ranks[t] = np.asarray(U[int(tr["lo"][t])]).shape[1]
            elif t == 0:
                transfer[t] = torch.from_numpy(np.ascontiguousarray(B[0], dtype=np.float64)).to(device)
            else:
                transfer[t] = torch.from_numpy(np.ascontiguousarray(B[t])).to(device=device, dtype=tdt)
                ranks[t] = np.asarray(B[t]).shape[0]
        n = [np.asarray(u).shape[0] for u in U]
        return DeviceHT(d, n, ranks, leaves, transfer, log2_scale)

    # -- views
    def scale_value(self) -> int:
        s = self.log2_scale
        return int(s.item()) if hasattr(s, "item") else int(s)

    def desc(self) -> HtDesc:
        import torch
        nn = 2 * self.d - 1
        n = (ctypes.c_int64 * self.d)(*self.n)
        rk = (ctypes.c_int32 * nn)(*self.ranks)
        leaf = (ctypes.c_void_p * self.d)(*[u.data_ptr() for u in self.leaves])
        ld = (ctypes.c_int64 * self.d)(*[u.shape[1] for u in self.leaves])
        tp = (ctypes.c_void_p * nn)(*[(b.data_ptr() if b is not None else 0) for b in self.transfer])
        for u in self.leaves:
            if not u.is_contiguous():
                raise HTError("leaf frames must be contiguous (k, n) tensors")
        inner = [b for t, b in enumerate(self.transfer) if b is not None and t != 0]
        tdt = _dt(inner[0].dtype) if inner else HT_F64
        desc = HtDesc(self.d, ctypes.cast(n, ctypes.POINTER(ctypes.c_int64)),
                      ctypes.cast(rk, ctypes.POINTER(ctypes.c_int32)), _dt(self.leaves[0].dtype), tdt,
                      ctypes.cast(leaf, ctypes.POINTER(ctypes.c_void_p)),
                      ctypes.cast(ld, ctypes.POINTER(ctypes.c_int64)),
                      ctypes.cast(tp, ctypes.POINTER(ctypes.c_void_p)), self.scale_value())
        desc._keep = (n, rk, leaf, ld, tp)
        return desc

    def to_host(self):
        """(U list of n x k float64, B dict, log2_scale) on the host."""
        U = [u.detach().double().cpu().numpy().T.copy() for u in self.leaves]
        B = {t: b.detach().double().cpu().numpy() for t, b in enumerate(self.transfer) if b is not None}
        return U, B, self.scale_value()


def _descs(xs: Sequence[DeviceHT]):
    arr = (HtDesc * len(xs))()
    keep = []
    for i, x in enumerate(xs):
        d = x.desc()
        arr[i] = d
        keep.append(d)
    return arr, keep


def _ws(nbytes, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------- operations
def ht_add(A: DeviceHT, C: DeviceHT, alpha=1.0, beta=1.0, S: Optional[DeviceHT] = None, ctx=None,
           stream=None) -> DeviceHT:
    """S = alpha A + beta C by Lemma (sum) (materialised)."""
    ctx = ctx or ht_create_context()
    if S is None:
        ranks = [a + c for a, c in zip(A.ranks, C.ranks)]
        S = DeviceHT.empty(A.d, A.n, ranks, A.leaves[0].dtype,
                           next(b for t, b in enumerate(A.transfer) if b is not None and t != 0).dtype
                           if A.d > 2 else None)
    s = ctypes.c_int64(0)
    da, db, ds = A.desc(), C.desc(), S.desc()
    _check(lib().ht_add(ctx.h, alpha, ctypes.byref(da), beta, ctypes.byref(db), ctypes.byref(ds),
                        ctypes.byref(s), _stream_ptr(stream)))
    S.log2_scale = int(s.value)
    return S


def ht_orthogonalize(X: DeviceHT, precision=HT_PREC_FP64, ctx=None, stream=None, ws=None):
    """In-place orthogonalisation (Section 3.4).  Returns (X, flags tensor)."""
    import torch
    ctx = ctx or ht_create_context()
    d = X.desc()
    need = ctypes.c_size_t(0)
    _check(lib().ht_orthogonalize_workspace(ctx.h, ctypes.byref(d), precision, ctypes.byref(need)))
    ws = ws if ws is not None and ws.numel() >= need.value else _ws(need.value)
    scale = torch.zeros(1, dtype=torch.int64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    _check(lib().ht_orthogonalize(ctx.h, ctypes.byref(d), precision, _ptr(scale), _ptr(flags), _ptr(ws),
                                  ws.numel(), _stream_ptr(stream)))
    X.log2_scale = scale
    return X, flags


def ht_gramians(X: DeviceHT, want_sigma=True, ctx=None, stream=None):
    """Reduced Gramians of an orthogonal tensor: (bhat list, sigma list, units tensor)."""
    import torch
    ctx = ctx or ht_create_context()
    nn = 2 * X.d - 1
    d = X.desc()
    need = ctypes.c_size_t(0)
    _check(lib().ht_gramians_workspace(ctx.h, ctypes.byref(d), ctypes.byref(need)))
    ws = _ws(need.value)
    bh = [None] + [torch.zeros((X.ranks[t], X.ranks[t]), dtype=torch.float64, device="cuda") for t in range(1, nn)]
    sg = [None] + [torch.zeros(X.ranks[t], dtype=torch.float64, device="cuda") for t in range(1, nn)]
    bp = (ctypes.c_void_p * nn)(*[(b.data_ptr() if b is not None else 0) for b in bh])
    sp = (ctypes.c_void_p * nn)(*[(s.data_ptr() if s is not None else 0) for s in sg])
    units = torch.zeros(1, dtype=torch.int64, device="cuda")
    _check(lib().ht_gramians(ctx.h, ctypes.byref(d), bp, sp if want_sigma else None, _ptr(units), _ptr(ws),
                             ws.numel(), _stream_ptr(stream)))
    return bh, (sg if want_sigma else None), units


class TruncResult:
    def __init__(self, out, ranks, scale, flags, sigma):
        self.out = out
        self.ranks_dev = ranks
        self.scale_dev = scale
        self.flags_dev = flags
        self.sigma_dev = sigma

    @property
    def ranks(self):
        return [int(x) for x in self.ranks_dev.cpu().numpy()]

    @property
    def flags(self):
        return int(self.flags_dev.item())


def out_ranks_for(Xs: Sequence[DeviceHT], mode, ranks=None, max_rank=0):
    """Output buffer ranks: fixed ranks clamped to the sum rank, or the
    tolerance-mode upper bound min(K_t, max_rank) (shared at the root sons)."""
    K = [sum(x.ranks[t] for x in Xs) for t in range(len(Xs[0].ranks))]
    K[0] = 1
    tr = ht_tree(Xs[0].d)
    out = [1] * len(K)
    for t in range(1, len(K)):
        if mode == HT_RANK_FIXED:
            out[t] = min(int(ranks[t]), K[t])
        else:
            out[t] = min(K[t], max_rank) if max_rank > 0 else K[t]
    if mode == HT_RANK_TOL:
        s1, s2 = int(tr["son1"][0]), int(tr["son2"][0])
        out[s1] = out[s2] = min(out[s1], out[s2])
    return out


class Truncator:
    """Reusable ht_truncate call: allocates output, workspace and the option
    structs once; __call__ enqueues one truncation on the current stream."""

    def __init__(self, Xs: Sequence[DeviceHT], coef=None, *, mode=HT_RANK_FIXED, ranks=None, eps=0.0,
                 relative=True, max_rank=0, precision=HT_PREC_MIXED, out_frame_dtype=None,
                 out_transfer_dtype=None, want_sigma=False, noalloc=False, ctx=None):
        import torch
        self.ctx = ctx or ht_create_context()
        self.noalloc = bool(noalloc)   # ht_truncate_noalloc: no workspace, the library's static scratch
        self.Xs = list(Xs)
        d = Xs[0].d
        nn = 2 * d - 1
        self.coef = (ctypes.c_double * len(Xs))(*([1.0] * len(Xs) if coef is None else list(coef)))
        rk = list(ranks) if ranks is not None else [1] * nn
        self._rk = (ctypes.c_int32 * nn)(*rk)
        self.opts = HtTruncOpts(mode, ctypes.cast(self._rk, ctypes.POINTER(ctypes.c_int32)), float(eps),
                                1 if relative else 0, int(max_rank), precision)
        fdt = out_frame_dtype or (torch.float32 if precision == HT_PREC_MIXED else torch.float64)
        tdt = out_transfer_dtype or fdt
        oranks = out_ranks_for(Xs, mode, rk, max_rank)
        self.out = DeviceHT.empty(d, Xs[0].n, oranks, fdt, tdt)
        self.xdescs, self._keep = _descs(self.Xs)
        need = ctypes.c_size_t(0)
        _check(lib().ht_truncate_workspace(self.ctx.h, self.xdescs, len(Xs), ctypes.byref(self.opts),
                                           ctypes.byref(need)))
        self.ws = None if self.noalloc else _ws(need.value)
        self.ws_bytes = need.value
        self.ranks = torch.zeros(nn, dtype=torch.int32, device="cuda")
        self.scale = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.flags = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.sigma = torch.zeros((nn, KMAX), dtype=torch.float64, device="cuda") if want_sigma else None
        self.odesc = self.out.desc()

    def __call__(self, stream=None):
        if self.noalloc:
            _check(lib().ht_truncate_noalloc(self.ctx.h, self.xdescs, self.coef, len(self.Xs),
                                             ctypes.byref(self.opts), ctypes.byref(self.odesc), _ptr(self.ranks),
                                             _ptr(self.scale), _ptr(self.flags), _ptr(self.sigma),
                                             _stream_ptr(stream)))
        else:
            _check(lib().ht_truncate(self.ctx.h, self.xdescs, self.coef, len(self.Xs), ctypes.byref(self.opts),
                                     ctypes.byref(self.odesc), _ptr(self.ranks), _ptr(self.scale),
                                     _ptr(self.flags), _ptr(self.sigma), _ptr(self.ws), self.ws_bytes,
                                     _stream_ptr(stream)))
        self.out.log2_scale = self.scale
        return TruncResult(self.out, self.ranks, self.scale, self.flags, self.sigma)


def ht_truncate(Xs, coef=None, **kw) -> TruncResult:
    """Truncate sum_c coef[c] Xs[c] (Section 3.3).  Keywords as Truncator."""
    if isinstance(Xs, DeviceHT):
        Xs = [Xs]
    return Truncator(Xs, coef, **kw)()


class BatchTruncator:
    """Reusable ht_truncate_batched call over independent problems.

    problems: list of dicts with keys ``Xs`` (summands, a list of DeviceHT),
    optional ``coef`` and the Truncator keywords ``mode``, ``ranks``, ``eps``,
    ``relative``, ``max_rank``, ``precision``, ``out_frame_dtype``,
    ``out_transfer_dtype``.  __call__ enqueues every truncation on the current
    stream and returns one TruncResult per problem."""

    def __init__(self, problems, *, want_sigma=False, ctx=None):
        import torch
        self.ctx = ctx or ht_create_context()
        self.count = len(problems)
        if self.count < 1:
            raise HTError("no problems")
        allx, coef, n_in = [], [], []
        self.opts = (HtTruncOpts * self.count)()
        self._rks, self.outs = [], []
        for c, pb in enumerate(problems):
            Xs = list(pb["Xs"])
            d = Xs[0].d
            nn = 2 * d - 1
            allx += Xs
            n_in.append(len(Xs))
            coef += [1.0] * len(Xs) if pb.get("coef") is None else [float(v) for v in pb["coef"]]
            mode = pb.get("mode", HT_RANK_FIXED)
            rk = list(pb["ranks"]) if pb.get("ranks") is not None else [1] * nn
            rka = (ctypes.c_int32 * nn)(*rk)
            self._rks.append(rka)
            prec = pb.get("precision", HT_PREC_MIXED)
            max_rank = int(pb.get("max_rank", 0))
            self.opts[c] = HtTruncOpts(mode, ctypes.cast(rka, ctypes.POINTER(ctypes.c_int32)),
                                       float(pb.get("eps", 0.0)), 1 if pb.get("relative", True) else 0, max_rank,
                                       prec)
            fdt = pb.get("out_frame_dtype") or (torch.float32 if prec == HT_PREC_MIXED else torch.float64)
            tdt = pb.get("out_transfer_dtype") or fdt
            self.outs.append(DeviceHT.empty(d, Xs[0].n, out_ranks_for(Xs, mode, rk, max_rank), fdt, tdt))
        self.Xs = allx
        self.xdescs, self._keep = _descs(allx)
        self.n_in = (ctypes.c_int32 * self.count)(*n_in)
        self.coef = (ctypes.c_double * len(coef))(*coef)
        self.odescs, self._okeep = _descs(self.outs)
        need = ctypes.c_size_t(0)
        _check(lib().ht_truncate_batched_workspace(self.ctx.h, self.count, self.xdescs, self.n_in, self.opts,
                                                   ctypes.byref(need)))
        self.ws = _ws(need.value)
        self.ws_bytes = need.value
        self.ranks = [torch.zeros(2 * o.d - 1, dtype=torch.int32, device="cuda") for o in self.outs]
        self.scale = torch.zeros(self.count, dtype=torch.int64, device="cuda")
        self.flags = torch.zeros(self.count, dtype=torch.int32, device="cuda")
        self.sigma = ([torch.zeros((2 * o.d - 1, KMAX), dtype=torch.float64, device="cuda") for o in self.outs]
                      if want_sigma else None)
        self._rp = (ctypes.c_void_p * self.count)(*[r.data_ptr() for r in self.ranks])
        self._sp = (ctypes.c_void_p * self.count)(*[s.data_ptr() for s in self.sigma]) if want_sigma else None

    def __call__(self, stream=None):
        _check(lib().ht_truncate_batched(self.ctx.h, self.count, self.xdescs, self.n_in, self.coef, self.opts,
                                         self.odescs, self._rp, _ptr(self.scale), _ptr(self.flags), self._sp,
                                         _ptr(self.ws), self.ws_bytes, _stream_ptr(stream)))
        res = []
        for c, o in enumerate(self.outs):
            o.log2_scale = self.scale[c:c + 1]
            res.append(TruncResult(o, self.ranks[c], self.scale[c:c + 1], self.flags[c:c + 1],
                                   self.sigma[c] if self.sigma is not None else None))
        return res


def ht_truncate_batched(problems, **kw):
    """Truncate many independent sums in one pass (list of TruncResult)."""
    return BatchTruncator(problems, **kw)()


def ht_entries(X: DeviceHT, idx, ctx=None, stream=None):
    """Entries for an m x d int32 index tensor (device) -> float64 tensor."""
    import torch
    ctx = ctx or ht_create_context()
    idx = idx.to(device="cuda", dtype=torch.int32).contiguous()
    m = idx.shape[0]
    d = X.desc()
    need = ctypes.c_size_t(0)
    _check(lib().ht_entries_workspace(ctx.h, ctypes.byref(d), m, ctypes.byref(need)))
    ws = _ws(need.value)
    out = torch.empty(m, dtype=torch.float64, device="cuda")
    _check(lib().ht_entries(ctx.h, ctypes.byref(d), m, _ptr(idx), _ptr(out), _ptr(ws), ws.numel(),
                            _stream_ptr(stream)))
    return out


class Scaled:
    """A device result m * 2^e (m: float64 tensor, e: int64 tensor, one element each)."""

    def __init__(self, m, e, flags=None):
        self.m, self.e, self.flags_dev = m, e, flags

    def mantissa_exponent(self):
        return float(self.m.item()), int(self.e.item())

    def value(self) -> float:
        """As a Python float (inf or 0 outside the float64 range)."""
        m, e = self.mantissa_exponent()
        return float(np.ldexp(m, int(np.clip(e, -20000, 20000))))

    def log2_abs(self) -> float:
        m, e = self.mantissa_exponent()
        return float(np.log2(abs(m)) + e) if m != 0.0 else float("-inf")


class Inner:
    """Reusable ht_inner call: descriptors, workspace and result buffers are
    set up once; __call__ enqueues <X, Y> (Definition (phi)) on the stream."""

    def __init__(self, X: DeviceHT, Y: DeviceHT, ctx=None):
        import torch
        self.ctx = ctx or ht_create_context()
        self.X, self.Y = X, Y
        self.dx, self.dy = X.desc(), Y.desc()
        need = ctypes.c_size_t(0)
        _check(lib().ht_inner_workspace(self.ctx.h, ctypes.byref(self.dx), ctypes.byref(self.dy),
                                        ctypes.byref(need)))
        self.ws = _ws(need.value)
        self.m = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.e = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.flags = torch.zeros(1, dtype=torch.int32, device="cuda")

    def __call__(self, stream=None) -> Scaled:
        _check(lib().ht_inner(self.ctx.h, ctypes.byref(self.dx), ctypes.byref(self.dy), _ptr(self.m), _ptr(self.e),
                              _ptr(self.flags), _ptr(self.ws), self.ws.numel(), _stream_ptr(stream)))
        return Scaled(self.m, self.e, self.flags)


class Norm:
    """Reusable ht_norm call for the lazy sum sum_c coef[c] Xs[c]."""

    def __init__(self, Xs, coef=None, ctx=None):
        import torch
        self.ctx = ctx or ht_create_context()
        self.Xs = [Xs] if isinstance(Xs, DeviceHT) else list(Xs)
        self.arr, self._keep = _descs(self.Xs)
        self.cf = (ctypes.c_double * len(self.Xs))(*([1.0] * len(self.Xs) if coef is None else list(coef)))
        need = ctypes.c_size_t(0)
        _check(lib().ht_norm_workspace(self.ctx.h, self.arr, len(self.Xs), ctypes.byref(need)))
        self.ws = _ws(need.value)
        self.m = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.e = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.flags = torch.zeros(1, dtype=torch.int32, device="cuda")

    def __call__(self, stream=None) -> Scaled:
        _check(lib().ht_norm(self.ctx.h, self.arr, self.cf, len(self.Xs), _ptr(self.m), _ptr(self.e),
                             _ptr(self.flags), _ptr(self.ws), self.ws.numel(), _stream_ptr(stream)))
        return Scaled(self.m, self.e, self.flags)


def ht_inner(X: DeviceHT, Y: DeviceHT, ctx=None, stream=None) -> Scaled:
    """<X, Y> by Definition (phi) / Lemma (phi), enqueued on the current stream."""
    f = Inner(X, Y, ctx)
    res = f(stream)
    res._ws = f.ws
    return res


def ht_norm(Xs, coef=None, ctx=None, stream=None) -> Scaled:
    """||sum_c coef[c] Xs[c]|| through the orthogonalised lazy sum (Section 3.4);
    ht_norm([A, B], [1, -1]) is the difference norm."""
    f = Norm(Xs, coef, ctx)
    res = f(stream)
    res._ws = f.ws
    return res


def ht_apply(L: DeviceHT, A: DeviceHT, C: Optional[DeviceHT] = None, ctx=None, stream=None,
             frame_dtype=None, transfer_dtype=None) -> DeviceHT:
    """C = L A by Lemma (operator).  L's mode mu has n_mu^2 rows (column r of
    its leaf frame: the matrix W_{mu,r} row-major).  C is allocated with
    ranks k^L_t k^A_t unless given; its scale is the sum of the two scales."""
    ctx = ctx or ht_create_context()
    if C is None:
        ranks = [1] + [a * b for a, b in zip(L.ranks[1:], A.ranks[1:])]
        inner = [b for t, b in enumerate(A.transfer) if b is not None and t != 0]
        C = DeviceHT.empty(A.d, A.n, ranks, frame_dtype or A.leaves[0].dtype,
                           transfer_dtype or (inner[0].dtype if inner else None))
    dl, da, dc = L.desc(), A.desc(), C.desc()
    _check(lib().ht_apply(ctx.h, ctypes.byref(dl), ctypes.byref(da), ctypes.byref(dc), _stream_ptr(stream)))
    C.log2_scale = L.scale_value() + A.scale_value()
    return C


# ---------------------------------------------------------------- profiling
def profile_enable(on=True, ctx=None):
    ctx = ctx or ht_create_context()
    _check(lib().ht_profile_enable(ctx.h, 1 if on else 0))


def profile_reset(ctx=None):
    ctx = ctx or ht_create_context()
    _check(lib().ht_profile_reset(ctx.h))


def profile_read(ctx=None):
    """Per (step, kernel) totals of the launches timed with HIP events."""
    ctx = ctx or ht_create_context()
    n = ctypes.c_int32(0)
    _check(lib().ht_profile_read(ctx.h, 0, None, ctypes.byref(n)))
    arr = (HtProfileEntry * max(1, n.value))()
    _check(lib().ht_profile_read(ctx.h, n.value, arr, ctypes.byref(n)))
    return [dict(label=e.label.decode(), kernel=e.kernel.decode(), launches=int(e.launches), ms=float(e.ms),
                 flops=float(e.flops), bytes=float(e.bytes)) for e in arr[:n.value]]
