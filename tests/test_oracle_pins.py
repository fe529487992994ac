"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: the reference values come from
full-tensor SVDs (numpy.linalg.svd of explicit matricisations), closed forms,
the d=8 tree figure of Section 2, exact identities (Lemma (sum), A+A = 2A,
invariance under Lemma (transfer tensor transformation)) and error bounds.
"""
import math
import os

import numpy as np
import pytest

import htsynth as S
from oracle import brute as BF
from oracle import ht_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_ht(rng, d, n, ranks=None, kmax=4, scale=0):
    """Random HT tensor with (possibly non-uniform) ranks on the balanced tree."""
    tr = O.Tree(d)
    ns = [int(n)] * d if np.isscalar(n) else list(n)
    if ranks is None:
        ranks = [1] + [int(rng.integers(1, kmax + 1)) for _ in range(tr.n_nodes - 1)]
    U = [None] * d
    B = {}
    for t in range(tr.n_nodes):
        if tr.is_leaf(t):
            U[tr.mode(t)] = rng.standard_normal((ns[tr.mode(t)], ranks[t]))
        else:
            s1, s2 = tr.sons[t]
            shape = (ranks[s1], ranks[s2]) if t == 0 else (ranks[t], ranks[s1], ranks[s2])
            B[t] = rng.standard_normal(shape)
    return O.HT(tr, U, B, scale)


# --------------------------------------------------------------- tree
def test_tree_matches_figure_d8():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "tree_d8.txt")) if l.strip() and not l.startswith("#")]
    tr = O.Tree(8)
    assert tr.n_nodes == len(rows) == 15
    for t, (lo, hi, dep) in enumerate(rows):
        assert (tr.lo[t], tr.hi[t], tr.depth[t]) == (int(lo), int(hi), int(dep))


@pytest.mark.parametrize("d", list(range(2, 70)))
def test_tree_depth_and_split(d):
    tr = O.Tree(d)
    assert tr.n_nodes == 2 * d - 1
    assert max(tr.depth) == math.ceil(math.log2(d))          # depth(T_d) = ceil(log2 d)
    assert [tr.mode(tr.leaf_node[m]) for m in range(d)] == list(range(d))
    for t in range(tr.n_nodes):
        if tr.sons[t]:
            s1, s2 = tr.sons[t]
            mu, nu = tr.lo[t], tr.hi[t]
            assert (tr.lo[s1], tr.hi[s1]) == (mu, (mu + nu - 1) // 2)
            assert (tr.lo[s2], tr.hi[s2]) == ((mu + nu - 1) // 2 + 1, nu)


# --------------------------------------------------------------- full tensor, entries, storage
def test_full_rank_one_is_outer_product():
    """All ranks 1: the tensor is prod(B) * u_1 o u_2 o ... o u_d (closed form)."""
    rng = np.random.default_rng(0)
    for d in (2, 3, 5, 6):
        X = rand_ht(rng, d, [3, 4, 2, 3, 2, 3][:d], ranks=[1] * (2 * d - 1))
        ref = X.U[0][:, 0]
        for mu in range(1, d):
            ref = np.multiply.outer(ref, X.U[mu][:, 0])
        ref = ref * np.prod([float(np.ravel(b)[0]) for b in X.B.values()])
        np.testing.assert_allclose(O.full(X), ref, rtol=1e-13, atol=0)


def test_full_d4_single_network_contraction():
    """d=4: A = sum B_D[p,q] B_12[p,a,b] B_34[q,c,e] U1[:,a] U2[:,b] U3[:,c] U4[:,e]."""
    rng = np.random.default_rng(1)
    X = rand_ht(rng, 4, [3, 4, 2, 5], kmax=3)
    tr = X.tree
    t12, t34 = tr.sons[0]
    ref = np.einsum("pq,pab,qce,ia,jb,kc,le->ijkl", X.B[0], X.B[t12], X.B[t34],
                    X.U[0], X.U[1], X.U[2], X.U[3])
    np.testing.assert_allclose(O.full(X), ref, rtol=1e-12, atol=1e-12)


def test_entries_match_full():
    rng = np.random.default_rng(2)
    for d in (2, 3, 4, 5, 7):
        X = rand_ht(rng, d, 3, kmax=3, scale=5)
        A = O.full(X)
        idx = S.entry_indices(40, d, 3, seed=d)
        np.testing.assert_allclose(O.entries(X, idx), A[tuple(idx.T)], rtol=1e-12, atol=1e-12 * np.abs(A).max())


def test_storage_complexity():
    """dnk + (d-2)k^3 + k^2 stored numbers for uniform ranks (eq. storageComplexity)."""
    for d, n, k in [(4, 16, 4), (16, 1000, 32), (7, 5, 3)]:
        X = O.from_input(S.make_tensor(0, d, n, k))
        cnt = sum(u.size for u in X.U) + sum(b.size for b in X.B.values())
        assert cnt == d * n * k + (d - 2) * k ** 3 + k ** 2


# --------------------------------------------------------------- sum
def test_sum_lemma():
    rng = np.random.default_rng(3)
    for d in (2, 3, 4, 6):
        A = rand_ht(rng, d, 3, kmax=3, scale=2)
        C = rand_ht(rng, d, 3, kmax=2, scale=-3)
        S_ = O.add(A, C, 0.5, -2.0)
        np.testing.assert_allclose(O.full(S_), 0.5 * O.full(A) - 2.0 * O.full(C), rtol=1e-12,
                                   atol=1e-12 * np.abs(O.full(A)).max())
        assert S_.ranks()[1:] == [a + c for a, c in zip(A.ranks()[1:], C.ranks()[1:])]


# --------------------------------------------------------------- orthogonalisation
@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_orthogonalize_preserves_and_orthonormal(d):
    rng = np.random.default_rng(10 + d)
    X = rand_ht(rng, d, [4, 3, 5, 2, 3, 4][:d], kmax=4, scale=7)
    A = O.full(X)
    Xo = O.orthogonalize(X)
    np.testing.assert_allclose(O.full(Xo), A, rtol=1e-12, atol=1e-12 * np.abs(A).max())
    tr = Xo.tree
    for t in range(1, tr.n_nodes):
        if tr.is_leaf(t):
            U = Xo.U[tr.mode(t)]
            np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)
        else:
            M23 = Xo.B[t].reshape(Xo.B[t].shape[0], -1).T
            np.testing.assert_allclose(M23.T @ M23, np.eye(M23.shape[1]), atol=1e-13)
    # ||A|| = ||B_D||_F 2^scale for an orthogonal tensor
    m, e = O.norm_log2(X)
    assert abs(np.ldexp(m, e) - np.linalg.norm(A)) <= 1e-13 * np.linalg.norm(A)


def test_orthogonalize_huge_scale():
    """Power-of-two scale tracking: entries far beyond float64 range keep exact mantissas."""
    rng = np.random.default_rng(5)
    X = rand_ht(rng, 4, 3, kmax=3)
    Y = X.copy()
    Y.log2_scale = 2000
    m0, e0 = O.norm_log2(X)
    m1, e1 = O.norm_log2(Y)
    assert e1 - e0 == 2000 and abs(m1 - m0) <= 1e-15


# --------------------------------------------------------------- Gramians
@pytest.mark.parametrize("d,n,kmax", [(2, 5, 4), (3, 4, 3), (4, 3, 4), (5, 3, 3), (6, 2, 3)])
def test_gramian_eigenvalues_are_singular_values(d, n, kmax):
    """sqrt(eig(Bhat_t)) = singular values of M_t(A) for every non-root t (Section 3.3)."""
    rng = np.random.default_rng(20 + d)
    X = rand_ht(rng, d, n, kmax=kmax, scale=3)
    A = O.full(X)
    Xo = O.orthogonalize(X)
    G, g = O.gramians(Xo)
    tr = X.tree
    for t in range(1, tr.n_nodes):
        lam, _ = O.eig_desc(G[t])
        sig = np.ldexp(np.sqrt(lam), g)
        sv = BF.singular_values(A, tr.modes(t))
        k = min(len(sig), len(sv))
        # the Gramian route squares: eigenvalues carry an absolute error of
        # order u * sigma_1^2, so compare sigma^2 (Section 5 notes this loss)
        np.testing.assert_allclose(sig[:k] ** 2, sv[:k] ** 2, atol=1e-12 * sv[0] ** 2)
        # trace(Bhat_t) = ||A||^2
        assert abs(np.ldexp(np.trace(G[t]), 2 * g) - np.sum(A * A)) <= 1e-12 * np.sum(A * A)


def test_gramian_eigenvectors_span_leading_singular_subspace():
    rng = np.random.default_rng(31)
    X = rand_ht(rng, 4, 4, ranks=[1, 3, 3, 3, 3, 3, 3])
    A = O.full(X)
    Xo = O.orthogonalize(X)
    G, _ = O.gramians(Xo)
    tr = X.tree
    for t in [tr.leaf_node[0], tr.leaf_node[3]]:
        _, Q = O.eig_desc(G[t])
        Ul = Xo.U[tr.mode(t)] @ Q[:, :2]                      # U_t Q_t = left singular vectors
        Ur = BF.leading_vectors(A, tr.modes(t), 2)
        np.testing.assert_allclose(Ul @ Ul.T, Ur @ Ur.T, atol=1e-11)


# --------------------------------------------------------------- truncation
@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_truncation_equals_root_first_projections(d):
    rng = np.random.default_rng(40 + d)
    X = rand_ht(rng, d, 3, kmax=4)
    C = rand_ht(rng, d, 3, kmax=3)
    Y = O.add(X, C)
    A = O.full(Y)
    tr = Y.tree
    kt = Y.ranks()
    ranks = [1] + [max(1, min(kt[t], BF.matricize(A, tr.modes(t)).shape[0]) - 1) for t in range(1, tr.n_nodes)]
    T, info = O.truncate(Y, mode="fixed", ranks=ranks)
    r = info["ranks"]
    P = BF.project_root_first(A, tr, r)
    np.testing.assert_allclose(O.full(T), P, atol=1e-11 * np.abs(A).max())
    H = BF.hsvd_full(A, tr, r)                                 # the paper's full-tensor HSVD
    np.testing.assert_allclose(O.full(H), P, atol=1e-11 * np.abs(A).max())


def test_projection_order_matters():
    """Applying the leaf projectors first gives a different tensor, so the
    root-first pin above discriminates the order."""
    rng = np.random.default_rng(50)
    Y = rand_ht(rng, 4, 4, ranks=[1, 4, 4, 4, 4, 4, 4])
    A = O.full(Y)
    tr = Y.tree
    r = {t: 2 for t in range(1, tr.n_nodes)}
    P_root = BF.project_root_first(A, tr, r)
    Pm = {t: BF.leading_vectors(A, tr.modes(t), 2) for t in range(1, tr.n_nodes)}
    X = A.copy()
    for depth in (2, 1):
        for t in range(1, tr.n_nodes):
            if tr.depth[t] == depth:
                M = BF.matricize(X, tr.modes(t))
                X = BF.unmatricize(Pm[t] @ (Pm[t].T @ M), tr.modes(t), A.shape)
    assert np.linalg.norm(X - P_root) > 1e-3 * np.linalg.norm(A)


def test_a_plus_a_is_2a():
    a, _ = S.workload_pair("d4_n16_k4")
    A = O.from_input(a)
    T, info = O.truncate(O.add(A, A), mode="fixed", ranks=[4] * 7)
    assert O.rel_diff(T, O.add(A, A, 2.0, 0.0)) < 1e-13
    assert all(v == 4 for v in info["ranks"].values())


def test_zero_partner_and_full_rank_identity():
    a, c = S.workload_pair("d4_n16_k4")
    A, C = O.from_input(a), O.from_input(c)
    T, _ = O.truncate(O.add(A, C, 1.0, 0.0), mode="fixed", ranks=[4] * 7)
    assert O.rel_diff(T, A) < 1e-13
    X = O.add(A, C)
    T, _ = O.truncate(X, mode="fixed", ranks=[8] * 7)
    assert O.rel_diff(T, X) < 1e-13


def test_d2_is_truncated_matrix_svd():
    """d = 2: the tensor is the matrix M = U1 B_D U2^T; truncation is Eckart-Young."""
    rng = np.random.default_rng(60)
    X = rand_ht(rng, 2, [9, 7], ranks=[1, 5, 6])
    M = X.U[0] @ X.B[0] @ X.U[1].T
    for r in (1, 2, 4):
        T, _ = O.truncate(X, mode="fixed", ranks=[1, r, r])
        U, s, Vt = np.linalg.svd(M)
        ref = (U[:, :r] * s[:r]) @ Vt[:r]
        np.testing.assert_allclose(O.full(T), ref, atol=1e-12 * s[0])


@pytest.mark.parametrize("d", [3, 4, 5, 6])
def test_error_sandwich(d):
    """max_t tau_t <= ||A - T(A)|| <= sqrt(sum over 2d-3 nodes tau_t^2) <= sqrt(2d-3) max_t tau_t."""
    rng = np.random.default_rng(70 + d)
    Y = O.add(rand_ht(rng, d, 3, kmax=3), rand_ht(rng, d, 3, kmax=3))
    A = O.full(Y)
    tr = Y.tree
    r = {t: 2 for t in range(1, tr.n_nodes)}
    T, info = O.truncate(Y, mode="fixed", ranks=[1] + [2] * (tr.n_nodes - 1))
    err = np.linalg.norm(O.full(T) - A)
    tau2 = {t: float(np.sum(BF.singular_values(A, tr.modes(t))[2:] ** 2)) for t in range(1, tr.n_nodes)}
    t2 = tr.sons[0][1]
    upper = math.sqrt(sum(v for t, v in tau2.items() if t != t2))
    lower = BF.best_error_lower_bound(A, tr, r)
    assert lower <= err * (1 + 1e-12)
    assert err <= upper * (1 + 1e-12)
    assert upper <= math.sqrt(2 * d - 3) * lower * (1 + 1e-12)


def test_tolerance_rule():
    rng = np.random.default_rng(80)
    Y = O.add(rand_ht(rng, 5, 4, kmax=4), rand_ht(rng, 5, 4, kmax=4))
    A = O.full(Y)
    nA = np.linalg.norm(A)
    for eps in (0.5, 0.1, 1e-2, 1e-4):
        T, info = O.truncate(Y, mode="tol", eps=eps)
        assert np.linalg.norm(O.full(T) - A) <= eps * nA * (1 + 1e-10)
        # minimality of each node's rank under the rule
        d = Y.d
        thr = (eps * nA) ** 2 / (2 * d - 3)
        for t, r in info["ranks"].items():
            sv = BF.singular_values(A, Y.tree.modes(t))
            if r > 1 and t not in Y.tree.sons[0]:
                assert np.sum(sv[r - 1:] ** 2) > thr * (1 - 1e-9)
    T, info = O.truncate(Y, mode="tol", eps=2.0)
    assert all(r == 1 for r in info["ranks"].values())
    T, info = O.truncate(Y, mode="tol", eps=0.0)
    assert O.rel_diff(T, Y) < 1e-12
    T, info = O.truncate(Y, mode="tol", eps=0.0, max_rank=2)
    assert all(r <= 2 for r in info["ranks"].values())


def test_absolute_tolerance_with_large_scale():
    rng = np.random.default_rng(81)
    Y = O.add(rand_ht(rng, 4, 4, kmax=3), rand_ht(rng, 4, 4, kmax=3))
    A = O.full(Y)
    eps = 0.05 * np.linalg.norm(A)
    T0, i0 = O.truncate(Y, mode="tol", eps=eps, relative=False)
    Z = Y.copy()
    Z.log2_scale += 900
    T1, i1 = O.truncate(Z, mode="tol", eps=np.ldexp(eps, 900), relative=False)
    assert i0["ranks"] == i1["ranks"]
    assert T1.log2_scale - T0.log2_scale == 900


# --------------------------------------------------------------- gauge invariance (Lemma transfer tensor transformation)
def test_gauge_invariance():
    rng = np.random.default_rng(90)
    Y = O.add(rand_ht(rng, 5, 3, kmax=3), rand_ht(rng, 5, 3, kmax=3))
    A = O.full(Y)
    tr = Y.tree
    Z = Y.copy()
    G = {t: rng.standard_normal((Y.rank(t), Y.rank(t))) + 3 * np.eye(Y.rank(t)) for t in range(1, tr.n_nodes)}
    for t in range(tr.n_nodes):
        if tr.is_leaf(t):
            Z.U[tr.mode(t)] = Y.U[tr.mode(t)] @ G[t]
        elif t == 0:
            s1, s2 = tr.sons[0]
            Z.B[0] = np.linalg.inv(G[s1]) @ Y.B[0] @ np.linalg.inv(G[s2]).T
        else:
            s1, s2 = tr.sons[t]
            B = O.mode_product(Y.B[t], G[t].T, 0)
            B = O.mode_product(B, np.linalg.inv(G[s1]), 1)
            Z.B[t] = O.mode_product(B, np.linalg.inv(G[s2]), 2)
    np.testing.assert_allclose(O.full(Z), A, atol=1e-10 * np.abs(A).max())
    r = [1] + [2] * (tr.n_nodes - 1)
    T0, _ = O.truncate(Y, mode="fixed", ranks=r)
    T1, _ = O.truncate(Z, mode="fixed", ranks=r)
    assert O.rel_diff(T1, T0) < 1e-10


# --------------------------------------------------------------- inner product (Section 3.2)
def test_inner_product_phi():
    rng = np.random.default_rng(100)
    for d in (2, 3, 4, 6):
        A = rand_ht(rng, d, 3, kmax=3, scale=1)
        C = rand_ht(rng, d, 3, kmax=4, scale=-2)
        ref = float(np.sum(O.full(A) * O.full(C)))
        assert abs(O.inner(A, C) - ref) <= 1e-12 * np.linalg.norm(O.full(A)) * np.linalg.norm(O.full(C))


def test_diff_norm_resolves_tiny_differences():
    """rel_diff via the orthogonalised difference sees 1e-12 relative changes
    that ||X||^2 + ||Y||^2 - 2<X,Y> cannot."""
    rng = np.random.default_rng(110)
    X = rand_ht(rng, 4, 4, kmax=3)
    Y = X.copy()
    Y.B[0] = Y.B[0] * (1 + 1e-12)
    rd = O.rel_diff(Y, X)
    assert 5e-13 < rd < 2e-12


# --------------------------------------------------------------- planted mistakes must be caught
def test_planted_mistake_wrong_son_gramian_is_caught(monkeypatch):
    """Swapping the contracted indices of eq. (acctransferSon1) breaks the
    singular-value pin."""
    rng = np.random.default_rng(120)
    X = rand_ht(rng, 4, 3, ranks=[1, 3, 3, 3, 3, 3, 3])
    A = O.full(X)
    Xo = O.orthogonalize(X)
    real = np.einsum

    def bad(expr, *ops, **kw):
        if expr == "ipl,ij,jql->pq":
            expr = "ilp,ij,jlq->pq"
        return real(expr, *ops, **kw)
    monkeypatch.setattr(O.np, "einsum", bad)
    G, g = O.gramians(Xo)
    monkeypatch.setattr(O.np, "einsum", real)
    tr = X.tree
    t12 = tr.sons[0][0]
    s1 = tr.sons[t12][0]
    lam, _ = O.eig_desc(G[s1])
    sv = BF.singular_values(A, tr.modes(s1))
    assert np.max(np.abs(np.ldexp(np.sqrt(lam), g) - sv[:3])) > 1e-6 * sv[0]


def test_planted_mistake_dropped_r_is_caught(monkeypatch):
    """Skipping the R_s2 update of the father in the orthogonalisation changes the tensor."""
    rng = np.random.default_rng(121)
    X = rand_ht(rng, 4, 3, kmax=3)
    A = O.full(X)
    real = O.mode_product
    calls = {"n": 0}

    def bad(B, M, axis):
        if axis == 2 and M.shape[0] == M.shape[1] and B.ndim == 3:
            calls["n"] += 1
            return B
        return real(B, M, axis)
    monkeypatch.setattr(O, "mode_product", bad)
    Xo = O.orthogonalize(X)
    monkeypatch.setattr(O, "mode_product", real)
    assert calls["n"] > 0
    assert np.linalg.norm(O.full(Xo) - A) > 1e-3 * np.linalg.norm(A)
