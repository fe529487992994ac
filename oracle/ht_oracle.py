"""Plain FP64 CPU oracle for truncating Hierarchical Tucker (HT) tensors and
their sums by the hierarchical SVD.

TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
the test-suite, the smoke check and the benchmark's CPU-baseline leg import
it.  It shares no code with the HIP path (no kernels, headers, helpers or
constants) and must never be called by the library.

Everything is float64 NumPy.  Library primitives used as single steps:
``numpy.linalg.qr`` (Householder reduced QR), ``numpy.linalg.eigh``
(symmetric eigensolver), ``tensordot``/``einsum`` (contractions).  Each
function follows the passage of the paper it cites (Grasedyck & Loebbert,
"Distributed Hierarchical SVD in the Hierarchical Tucker Format"):

* dimension tree ...................... Section 2, eq. (balanced)
* HT format, transfer tensors ......... Section 2.1, eq. (transfer)
* entry evaluation .................... Section 3.1, eq. (transfermult) and the root formula
* inner product ....................... Section 3.2, Definition (Phi), eq. (defphi), Lemma (phi)
* Gramians, truncation ................ Section 3.3, eqs. (acctransferroot), (acctransferSon1/2),
                                        (nodewisetruncation), (transfertransformationtrunc)
* orthogonalisation ................... Section 3.4, eq. (qrtransfer) and the three-step algorithm
* sum ................................. Section 3.5, Lemma (sum)

Readings where the paper is silent (all listed in the design notes):

* power-of-two scale tracking: every R factor is divided by 2^e, with e the
  binary exponent of its largest entry, and e is added to ``log2_scale``;
  the represented tensor is 2^log2_scale times the stored one;
* the tolerance rank rule: r_t = min{ r >= 1 : sum_{i>r} lambda_{t,i} <=
  eps_abs^2 / (2d-3) }, capped by max_rank and k_t; the two sons of the root
  share one rank, computed from the first son;
* Kronecker order: in (U_s1 (x) U_s2) the index of s1 runs slowest, and the
  full tensor is stored C-order (mode 1 slowest).
"""
from __future__ import annotations

import copy
from typing import Dict, List, Optional

import numpy as np

__all__ = [
    "Tree", "HT", "from_input", "full", "entries", "add", "orthogonalize",
    "gramians", "eig_desc", "select_ranks", "truncate", "inner", "norm_log2",
    "diff_norm_log2", "rel_diff", "mode_product",
]


# --------------------------------------------------------------------------
# Dimension tree -- Section 2, eq. (balanced)
# --------------------------------------------------------------------------
class Tree:
    """Balanced dimension tree T_d.  A node {mu..nu} (1-based modes) has the
    sons {mu .. floor((mu+nu-1)/2)} and {floor((mu+nu-1)/2)+1 .. nu}.
    Nodes are numbered in preorder: root 0, then the first son's subtree,
    then the second son's subtree."""

    def __init__(self, d: int):
        if d < 2:
            raise ValueError("d must be >= 2")
        self.d = d
        self.lo: List[int] = []      # 1-based first mode of the node
        self.hi: List[int] = []      # 1-based last mode
        self.sons: List[Optional[tuple]] = []
        self.parent: List[int] = []
        self.depth: List[int] = []
        self._visit(1, d, -1, 0)
        self.n_nodes = len(self.lo)
        self.height = [0] * self.n_nodes
        for t in reversed(range(self.n_nodes)):
            if self.sons[t] is not None:
                s1, s2 = self.sons[t]
                self.height[t] = 1 + max(self.height[s1], self.height[s2])
        self.leaf_node = [0] * d      # mode (0-based) -> node id
        for t in range(self.n_nodes):
            if self.sons[t] is None:
                self.leaf_node[self.lo[t] - 1] = t

    def _visit(self, mu, nu, parent, depth):
        t = len(self.lo)
        self.lo.append(mu)
        self.hi.append(nu)
        self.parent.append(parent)
        self.depth.append(depth)
        self.sons.append(None)
        if mu < nu:
            split = (mu + nu - 1) // 2
            s1 = self._visit(mu, split, t, depth + 1)
            s2 = self._visit(split + 1, nu, t, depth + 1)
            self.sons[t] = (s1, s2)
        return t

    def is_leaf(self, t):
        return self.sons[t] is None

    def mode(self, t):
        """0-based mode of a leaf node."""
        return self.lo[t] - 1

    def modes(self, t):
        """0-based modes of node t."""
        return list(range(self.lo[t] - 1, self.hi[t]))

    def inner_nonroot(self):
        return [t for t in range(1, self.n_nodes) if not self.is_leaf(t)]

    def postorder(self):
        out = []

        def rec(t):
            if self.sons[t] is not None:
                rec(self.sons[t][0])
                rec(self.sons[t][1])
            out.append(t)
        rec(0)
        return out


# --------------------------------------------------------------------------
# HT tensor -- Section 2.1
# --------------------------------------------------------------------------
class HT:
    """HT tensor: leaf frames U[mu] (n_mu x k_mu), transfer tensors B[t]
    (k_t x k_s1 x k_s2) for inner non-root t, root matrix B[0] (k_t1 x k_t2).
    The represented tensor is 2^log2_scale times the one the data spells out."""

    def __init__(self, tree: Tree, U: List[np.ndarray], B: Dict[int, np.ndarray], log2_scale: int = 0):
        self.tree = tree
        self.U = [np.asarray(u, dtype=np.float64) for u in U]
        self.B = {t: np.asarray(b, dtype=np.float64) for t, b in B.items()}
        self.log2_scale = int(log2_scale)

    @property
    def d(self):
        return self.tree.d

    @property
    def n(self):
        return [u.shape[0] for u in self.U]

    def rank(self, t):
        if t == 0:
            return 1
        if self.tree.is_leaf(t):
            return self.U[self.tree.mode(t)].shape[1]
        return self.B[t].shape[0]

    def ranks(self):
        return [self.rank(t) for t in range(self.tree.n_nodes)]

    def copy(self):
        return HT(self.tree, [u.copy() for u in self.U], {t: b.copy() for t, b in self.B.items()},
                  self.log2_scale)


def from_input(inp) -> HT:
    """Wrap a generated input: inner[j] belongs to the j-th non-root inner
    node in preorder."""
    tree = Tree(inp.d)
    B = {0: np.asarray(inp.root, dtype=np.float64)}
    for j, t in enumerate(tree.inner_nonroot()):
        B[t] = np.asarray(inp.inner[j], dtype=np.float64)
    return HT(tree, [np.asarray(u, dtype=np.float64) for u in inp.leaves], B, inp.log2_scale)


def mode_product(B: np.ndarray, M: np.ndarray, axis: int) -> np.ndarray:
    """Multiply tensor B along `axis` by matrix M: new[.., i, ..] = sum_m M[i, m] B[.., m, ..].
    (X, Y, Z) o B of Lemma (transfer tensor transformation) is mode_product
    applied with X on axis 0, Y on axis 1 and Z on axis 2."""
    out = np.tensordot(M, B, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def _as3(X: HT, t):
    """Transfer tensor of t as a 3-way array (the root gets k_D = 1)."""
    b = X.B[t]
    return b[None, :, :] if t == 0 else b


def _exp2(x: float) -> int:
    """Binary exponent e with x = m 2^e, 0.5 <= m < 1 (0 for x == 0)."""
    if x == 0.0 or not np.isfinite(x):
        return 0
    return int(np.frexp(x)[1])


# --------------------------------------------------------------------------
# Full tensor and entries -- Section 2.1 eq. (transfer), Section 3.1
# --------------------------------------------------------------------------
def _frame(X: HT, t):
    """Explicit frame U_t (rows: C-order over the modes of t) by eq. (transfer).
    Only for tiny tensors."""
    tr = X.tree
    if tr.is_leaf(t):
        return X.U[tr.mode(t)]
    s1, s2 = tr.sons[t]
    U1, U2 = _frame(X, s1), _frame(X, s2)
    B = _as3(X, t)
    Ut = np.einsum("qjl,aj,bl->abq", B, U1, U2)
    return Ut.reshape(U1.shape[0] * U2.shape[0], B.shape[0])


def full(X: HT) -> np.ndarray:
    """All n_1 x ... x n_d entries (mode 1 slowest).  Tiny tensors only."""
    col = _frame(X, 0)[:, 0]
    return np.ldexp(col, X.log2_scale).reshape(X.n)


def entries(X: HT, idx: np.ndarray) -> np.ndarray:
    """Entries A[i_1..i_d] for m multi-indices (m x d, 0-based) by the
    level-wise recursion of Section 3.1: leaves pick row i_mu, inner nodes
    apply eq. (transfermult), the root applies the root formula.  Row vectors
    are renormalised by powers of two per index (the exponents are summed)."""
    tr = X.tree
    idx = np.asarray(idx)
    m = idx.shape[0]
    rows: Dict[int, np.ndarray] = {}
    expo: Dict[int, np.ndarray] = {}
    for t in tr.postorder():
        if tr.is_leaf(t):
            y = X.U[tr.mode(t)][idx[:, tr.mode(t)], :]
            e = np.zeros(m, dtype=np.int64)
        else:
            s1, s2 = tr.sons[t]
            B = _as3(X, t)
            # (U_t)_{i_t, q} = sum_{j,l} (B_t)_{q,j,l} (U_s1)_{i_s1, j} (U_s2)_{i_s2, l},
            # the double sum taken as the sum over j (one matrix product) and
            # then the sum over l
            inner_j = np.tensordot(rows[s1], B, axes=([1], [1]))     # [m, q, l]
            y = np.einsum("mql,ml->mq", inner_j, rows[s2])
            e = expo[s1] + expo[s2]
        mx = np.max(np.abs(y), axis=1)
        ee = np.array([_exp2(v) for v in mx], dtype=np.int64)
        rows[t] = np.ldexp(y, -ee[:, None])
        expo[t] = e + ee
    val = rows[0][:, 0]
    return np.ldexp(val, (expo[0] + X.log2_scale).astype(np.int64))


# --------------------------------------------------------------------------
# Sum -- Section 3.5, Lemma (sum)
# --------------------------------------------------------------------------
def add(A: HT, C: HT, alpha: float = 1.0, beta: float = 1.0) -> HT:
    """alpha*A + beta*C by Lemma (sum): leaf frames side by side, inner
    transfer tensors block-diagonal (blocks (0,0,0) and (1,1,1)), root
    block-diagonal.  The coefficients and the scale difference go on the
    root blocks."""
    if A.d != C.d or A.n != C.n:
        raise ValueError("summands must share d and n")
    tr = A.tree
    s = max(A.log2_scale, C.log2_scale)
    a = np.ldexp(alpha, A.log2_scale - s)
    c = np.ldexp(beta, C.log2_scale - s)
    U = [np.hstack([A.U[mu], C.U[mu]]) for mu in range(A.d)]
    B = {}
    for t in range(tr.n_nodes):
        if tr.is_leaf(t):
            continue
        if t == 0:
            b, f = A.B[0], C.B[0]
            H = np.zeros((b.shape[0] + f.shape[0], b.shape[1] + f.shape[1]))
            H[:b.shape[0], :b.shape[1]] = a * b
            H[b.shape[0]:, b.shape[1]:] = c * f
        else:
            b, f = A.B[t], C.B[t]
            H = np.zeros(tuple(x + y for x, y in zip(b.shape, f.shape)))
            H[:b.shape[0], :b.shape[1], :b.shape[2]] = b
            H[b.shape[0]:, b.shape[1]:, b.shape[2]:] = f
        B[t] = H
    return HT(tr, U, B, s)


# --------------------------------------------------------------------------
# Orthogonalisation -- Section 3.4
# --------------------------------------------------------------------------
def orthogonalize(X: HT) -> HT:
    """Bottom-up orthogonalisation (Section 3.4, three-step algorithm):
    1. leaves: reduced QR U = Q R, U <- Q, R goes to the father;
    2. inner nodes: B <- (I, R_s1, R_s2) o B, reduced QR of M_{2,3}(B) as in
       eq. (qrtransfer), B_{q,j,l} <- Q_{(j,l),q}, R_t goes to the father;
    3. root: B_D <- R_t1 B_D R_t2^T.
    Sons are always processed before their father (post-order)."""
    tr = X.tree
    Y = X.copy()
    R: Dict[int, np.ndarray] = {}
    scale = Y.log2_scale
    for t in tr.postorder():
        if tr.is_leaf(t):
            mu = tr.mode(t)
            Q, Rt = np.linalg.qr(Y.U[mu], mode="reduced")
            Y.U[mu] = Q
        elif t != 0:
            s1, s2 = tr.sons[t]
            Bp = mode_product(mode_product(Y.B[t], R[s1], 1), R[s2], 2)
            kt, k1, k2 = Bp.shape
            M23 = Bp.reshape(kt, k1 * k2).T          # rows (j,l), j slowest; columns i
            Q, Rt = np.linalg.qr(M23, mode="reduced")
            Y.B[t] = Q.T.reshape(Q.shape[1], k1, k2)
        else:
            t1, t2 = tr.sons[0]
            Y.B[0] = R[t1] @ Y.B[0] @ R[t2].T
            continue
        e = _exp2(float(np.max(np.abs(Rt)))) if Rt.size else 0
        R[t] = np.ldexp(Rt, -e)
        scale += e
    Y.log2_scale = scale
    return Y


# --------------------------------------------------------------------------
# Gramians and eigenvectors -- Section 3.3
# --------------------------------------------------------------------------
def gramians(Xo: HT):
    """Reduced Gramians Bhat_t = V_t^T V_t of an orthogonal HT tensor for
    every non-root node: eq. (acctransferroot) at the sons of the root, then
    eqs. (acctransferSon1) and (acctransferSon2) top-down.

    Returned in units of 2^(2*g): the true Gramian is Bhat * 4^g with
    g = e_D + log2_scale, e_D the binary exponent of ||B_D||_F (B_D is
    divided by 2^e_D before the products so that trace(Bhat) is about 1)."""
    tr = Xo.tree
    BD = Xo.B[0]
    eD = _exp2(float(np.linalg.norm(BD)))
    BDn = np.ldexp(BD, -eD)
    G: Dict[int, np.ndarray] = {}
    t1, t2 = tr.sons[0]
    G[t1] = BDn @ BDn.T
    G[t2] = BDn.T @ BDn
    for t in range(1, tr.n_nodes):             # preorder: a father precedes its sons
        if tr.is_leaf(t):
            continue
        s1, s2 = tr.sons[t]
        B = Xo.B[t]
        Bh = G[t]
        G[s1] = np.einsum("ipl,ij,jql->pq", B, Bh, B, optimize=True)
        G[s2] = np.einsum("ijp,ik,kjq->pq", B, Bh, B, optimize=True)
    return G, eD + Xo.log2_scale


def eig_desc(Bh: np.ndarray):
    """Eigenpairs of a symmetric Gramian in descending order, eigenvalues
    clipped at 0 (Bhat Q = Q Sigma^2, Section 3.3)."""
    lam, Q = np.linalg.eigh(Bh)
    order = np.argsort(-lam, kind="stable")
    lam = np.maximum(lam[order], 0.0)
    return lam, Q[:, order]


def select_ranks(tree: Tree, lam: Dict[int, np.ndarray], kt: Dict[int, int], *, mode: str,
                 ranks=None, eps: float = 0.0, relative: bool = True, max_rank: int = 0,
                 norm_units: float = 1.0, eps_units_log2: int = 0):
    """Ranks r_t of every non-root node.

    mode "fixed": r_t = min(ranks[t], k_t).
    mode "tol":   r_t = min{ r >= 1 : sum_{i>r} lambda_i <= eps_abs^2/(2d-3) },
                  then min(r_t, max_rank, k_t); the sons of the root share
                  one rank.  eps_abs = eps*||A|| (relative) or eps (absolute).
    lambda are in the Gramian units of `gramians`; norm_units = ||A|| in
    those units (square root of the common trace) and eps_units_log2 = g."""
    d = tree.d
    r = {}
    t1, t2 = tree.sons[0]
    for t in range(1, tree.n_nodes):
        if mode == "fixed":
            r[t] = int(min(ranks[t], kt[t]))
            continue
        if relative:
            thr = (eps * norm_units) ** 2 / (2 * d - 3)
        else:
            e_n = np.ldexp(eps, -eps_units_log2)
            thr = e_n * e_n / (2 * d - 3)
        lt = lam[t]
        tail = np.concatenate([np.cumsum(lt[::-1])[::-1][1:], [0.0]])   # tail[r-1] = sum_{i>r}
        rr = len(lt)
        for cand in range(1, len(lt) + 1):
            if tail[cand - 1] <= thr:
                rr = cand
                break
        cap = kt[t] if max_rank <= 0 else min(max_rank, kt[t])
        r[t] = int(max(1, min(rr, cap)))
    if mode != "fixed":
        rr = min(r[t1], kt[t1], kt[t2])
        r[t1] = r[t2] = rr
    return r


def truncate(X: HT, *, mode: str = "fixed", ranks=None, eps: float = 0.0, relative: bool = True,
             max_rank: int = 0, already_orthogonal: bool = False):
    """Truncation by the hierarchical SVD (Section 3.3):
    orthogonalise (unless already orthogonal), compute all Gramians and their
    eigenvectors first, choose ranks, then apply eq. (nodewisetruncation) at
    the leaves, eq. (transfertransformationtrunc) at inner nodes and
    B_D <- Q_t1|^T B_D Q_t2| at the root.

    Returns (T, info) with info = dict(ranks, lam, sigma, gram_log2, norm)."""
    tr = X.tree
    Xo = X if already_orthogonal else orthogonalize(X)
    G, g = gramians(Xo)
    lam, Q = {}, {}
    for t in range(1, tr.n_nodes):
        lam[t], Q[t] = eig_desc(G[t])
    kt = {t: Xo.rank(t) for t in range(1, tr.n_nodes)}
    t1, _ = tr.sons[0]
    norm_units = float(np.sqrt(np.sum(lam[t1])))
    r = select_ranks(tr, lam, kt, mode=mode, ranks=ranks, eps=eps, relative=relative,
                     max_rank=max_rank, norm_units=norm_units, eps_units_log2=g)
    Qr = {t: Q[t][:, :r[t]] for t in range(1, tr.n_nodes)}
    T = Xo.copy()
    for t in range(tr.n_nodes):
        if tr.is_leaf(t):
            mu = tr.mode(t)
            T.U[mu] = Xo.U[mu] @ Qr[t]                       # eq. (nodewisetruncation)
        elif t != 0:
            s1, s2 = tr.sons[t]
            B = mode_product(Xo.B[t], Qr[t].T, 0)            # eq. (transfertransformationtrunc)
            B = mode_product(B, Qr[s1].T, 1)
            T.B[t] = mode_product(B, Qr[s2].T, 2)
        else:
            s1, s2 = tr.sons[0]
            T.B[0] = Qr[s1].T @ Xo.B[0] @ Qr[s2]
    # the result's root in units of 2^e, e the binary exponent of ||B_D||_F
    # of the orthogonalised tensor: an exact power-of-two rescaling that keeps
    # repeatedly truncated tensors (the iterates of Algorithms (CG) and
    # (richardson)) away from the floating-point range limits
    eD = _exp2(float(np.linalg.norm(Xo.B[0])))
    T.B[0] = np.ldexp(T.B[0], -eD)
    T.log2_scale += eD
    sigma = {t: np.sqrt(lam[t]) for t in lam}
    info = dict(ranks=r, lam=lam, sigma=sigma, gram_log2=g, norm_units=norm_units, Xo=Xo)
    return T, info


# --------------------------------------------------------------------------
# Inner product -- Section 3.2
# --------------------------------------------------------------------------
def inner(A: HT, C: HT) -> float:
    """<A, C> by Definition (Phi): Phi_mu = U_mu^T V_mu at the leaves,
    eq. (defphi) at inner nodes, <A,C> = Phi_D (Lemma (phi))."""
    tr = A.tree
    Phi: Dict[int, np.ndarray] = {}
    for t in tr.postorder():
        if tr.is_leaf(t):
            mu = tr.mode(t)
            Phi[t] = A.U[mu].T @ C.U[mu]
        else:
            s1, s2 = tr.sons[t]
            Bt, Ft = _as3(A, t), _as3(C, t)
            Phi[t] = np.einsum("abc,bd,ce,fde->af", Bt, Phi[s1], Phi[s2], Ft, optimize=True)
    return float(np.ldexp(Phi[0][0, 0], A.log2_scale + C.log2_scale))


def norm_log2(X: HT):
    """||X|| as (m, e) with ||X|| = m 2^e: ||B_D||_F after orthogonalisation
    (Section 3.4), which is exact for an orthogonal HT tensor."""
    Xo = orthogonalize(X)
    v = float(np.linalg.norm(Xo.B[0]))
    e = _exp2(v)
    return np.ldexp(v, -e), e + Xo.log2_scale


def diff_norm_log2(X: HT, Y: HT):
    """||X - Y|| as (m, e), from the orthogonalised HT difference X + (-1) Y.
    Unlike ||X||^2 + ||Y||^2 - 2<X,Y> it does not cancel."""
    return norm_log2(add(X, Y, 1.0, -1.0))


def rel_diff(X: HT, Y: HT) -> float:
    """||X - Y|| / ||Y||."""
    m1, e1 = diff_norm_log2(X, Y)
    m2, e2 = norm_log2(Y)
    if m2 == 0.0:
        return float("inf") if m1 else 0.0
    return float(np.ldexp(m1 / m2, e1 - e2))
