"""Operators in the HT format and the truncated iterative solvers built on
them (TEST INFRASTRUCTURE ONLY: like the rest of ``oracle/`` this is the
checker, never called by the library).

* ``apply``                 -- Lemma (operator), Section 3.6: C = L A with
                               transfer tensors F_t = H_t (x) B_t and leaf
                               frames V_mu[j, (r, l)] = sum_i W_mu[(j, i), r] U_mu[i, l];
* ``kron_sum_operator``     -- the H-operator of sum_mu I (x) .. (x) M_mu (x) .. (x) I
                               (hierarchical ranks 2), a synthetic SPD
                               operator when every M_mu is SPD;
* ``operator_matrix``       -- the full matrix of an H-operator (tiny sizes);
* ``cg``, ``cg_step``      -- Algorithm (CG): CG in HT arithmetic with a
                               truncation after every sum and every
                               operator application;
* ``richardson_step``, ``richardson`` -- Algorithm (richardson).

An H-operator is stored as an ``HT`` whose mode mu has n_mu^2 rows: column r
of leaf frame mu is the n_mu x n_mu matrix W_{mu,r}, entry (j, i) in row
j * n_mu + i (the index pair (j_mu, i_mu) of eq. (operatorastensor), the
row index j slowest).  In F_t = H_t (x) B_t the operator index runs slowest:
row (p, i) of F_t is p * k_t + i, and likewise for the columns (r, l) of the
leaf frames.
"""
from __future__ import annotations

from typing import Callable, Dict, List

import numpy as np

from .ht_oracle import HT, Tree, add, full, inner, truncate

__all__ = ["apply", "kron_sum_operator", "operator_matrix", "cg", "cg_step", "richardson_step", "richardson",
           "truncation"]


def apply(L: HT, A: HT) -> HT:
    """C = L A by Lemma (operator) (square operators: n_mu x n_mu matrices)."""
    tr = A.tree
    if L.d != A.d:
        raise ValueError("operator and tensor must share d")
    U = []
    for mu in range(A.d):
        n = A.U[mu].shape[0]
        W = L.U[mu]
        if W.shape[0] != n * n:
            raise ValueError("operator frame rows must be n_mu^2")
        kb = W.shape[1]
        W3 = W.reshape(n, n, kb)                       # [j, i, r]
        V = np.einsum("jir,il->jrl", W3, A.U[mu])     # column (r, l), r slowest
        U.append(V.reshape(n, kb * A.U[mu].shape[1]))
    B: Dict[int, np.ndarray] = {}
    for t in range(tr.n_nodes):
        if tr.is_leaf(t):
            continue
        H, Bt = L.B[t], A.B[t]
        if t == 0:
            F = np.einsum("qr,jl->qjrl", H, Bt)
            B[t] = F.reshape(H.shape[0] * Bt.shape[0], H.shape[1] * Bt.shape[1])
        else:
            F = np.einsum("pqr,ijl->piqjrl", H, Bt)
            B[t] = F.reshape(H.shape[0] * Bt.shape[0], H.shape[1] * Bt.shape[1], H.shape[2] * Bt.shape[2])
    return HT(tr, U, B, L.log2_scale + A.log2_scale)


def kron_sum_operator(mats: List[np.ndarray]) -> HT:
    """H-operator of sum_mu I (x) .. (x) M_mu (x) .. (x) I: leaf frames
    [vec(I), vec(M_mu)]; at every inner node column 0 of the frame is the
    identity on the node's modes and column 1 the sum of the terms with one
    M_mu among them, so H_t[0,0,0] = H_t[1,1,0] = H_t[1,0,1] = 1; the root
    adds the two sons' sums, B_D[1,0] = B_D[0,1] = 1."""
    d = len(mats)
    tr = Tree(d)
    U = []
    for M in mats:
        n = M.shape[0]
        U.append(np.stack([np.eye(n).reshape(-1), np.asarray(M, dtype=np.float64).reshape(-1)], axis=1))
    B: Dict[int, np.ndarray] = {}
    for t in range(tr.n_nodes):
        if tr.is_leaf(t):
            continue
        if t == 0:
            H = np.zeros((2, 2))
            H[1, 0] = H[0, 1] = 1.0
        else:
            H = np.zeros((2, 2, 2))
            H[0, 0, 0] = H[1, 1, 0] = H[1, 0, 1] = 1.0
        B[t] = H
    return HT(tr, U, B, 0)


def operator_matrix(L: HT, n: List[int]) -> np.ndarray:
    """The (prod n) x (prod n) matrix of an H-operator, rows (j_1..j_d) and
    columns (i_1..i_d) in C-order: eq. (operatorastensor) read backwards."""
    T = full(L)                                       # modes of size n_mu^2, index (j, i)
    d = len(n)
    T = T.reshape([x for m in n for x in (m, m)])     # j_1, i_1, j_2, i_2, ...
    T = np.transpose(T, [2 * m for m in range(d)] + [2 * m + 1 for m in range(d)])
    N = int(np.prod(n))
    return T.reshape(N, N)


def truncation(mode: str = "fixed", ranks=None, eps: float = 0.0, relative: bool = True) -> Callable[[HT], HT]:
    """The truncation T of the algorithms: to fixed ranks or to accuracy eps."""
    def T(X: HT) -> HT:
        r = None
        if mode == "fixed":
            r = [min(int(ranks[t]), X.rank(t)) if t else 1 for t in range(X.tree.n_nodes)]
        Y, _ = truncate(X, mode=mode, ranks=r, eps=eps, relative=relative)
        return Y
    return T


def cg(Aop: HT, B: HT, T: Callable[[HT], HT], eps: float, max_steps: int, history=None):
    """Algorithm (CG): X_0 = B, R_0 = T(B - A X_0), D_0 = R_0; while
    sqrt(<R_j, R_j>) > eps and j < max_steps: Z = T(A D_j),
    alpha = <R_j, R_j> / <D_j, Z>, X_j+1 = T(X_j + alpha D_j),
    R_j+1 = T(R_j - alpha Z), beta = <R_j+1, R_j+1> / <R_j, R_j>,
    D_j+1 = T(beta D_j + R_j+1).  Returns (X, number of steps)."""
    X = B
    R = T(add(B, apply(Aop, X), 1.0, -1.0))
    D = R
    rr = inner(R, R)
    j = 0
    while np.sqrt(max(rr, 0.0)) > eps and j < max_steps:
        X, R, D, rr_new, alpha, beta = cg_step(Aop, T, X, R, D, rr)
        rr = rr_new
        j += 1
        if history is not None:
            history.append(dict(X=X, R=R, D=D, rr=rr, alpha=alpha, beta=beta))
    return X, j


def cg_step(Aop: HT, T: Callable[[HT], HT], X: HT, R: HT, D: HT, rr: float):
    """One pass of the loop of Algorithm (CG) from the state (X, R, D) with
    rr = <R, R>: returns (X', R', D', <R', R'>, alpha, beta)."""
    Z = T(apply(Aop, D))
    alpha = rr / inner(D, Z)
    X = T(add(X, D, 1.0, alpha))
    R = T(add(R, Z, 1.0, -alpha))
    rr_new = inner(R, R)
    beta = rr_new / rr
    D = T(add(D, R, beta, 1.0))
    return X, R, D, rr_new, alpha, beta


def richardson_step(Aop: HT, X: HT, B: HT, omega: float, T: Callable[[HT], HT]) -> HT:
    """One step of Algorithm (richardson): Z = T(A X); Z = T(Z - B);
    X <- T(X - omega Z)."""
    Z = T(apply(Aop, X))
    Z = T(add(Z, B, 1.0, -1.0))
    return T(add(X, Z, 1.0, -omega))


def richardson(Aop: HT, X: HT, B: HT, omega: float, T: Callable[[HT], HT], steps: int) -> HT:
    for _ in range(steps):
        X = richardson_step(Aop, X, B, omega, T)
    return X
