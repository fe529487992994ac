"""Full-tensor brute force for tiny HT tensors (TEST INFRASTRUCTURE ONLY).

Independent of the Gramian route in ``ht_oracle``: everything here works on
the explicit n_1 x ... x n_d array with full SVDs of matricisations.

* ``matricize``      -- Definition (Matricization), Section 2.1;
* ``hsvd_full``      -- the hierarchical SVD of a full tensor, Section 3.3
                        (the three enumerated steps before the HT-format
                        version): leading left singular vectors of every
                        M_t(A), transfer tensors by inner products, root
                        matrix by the inner product with M_D(A);
* ``project_root_first`` -- the same result written as orthogonal projections
                        P_t = U_t U_t^T applied to A, nodes nearest the
                        root first, the leaves last.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from .ht_oracle import HT, Tree

__all__ = ["matricize", "unmatricize", "singular_values", "leading_vectors", "hsvd_full",
           "project_root_first", "best_error_lower_bound"]


def matricize(A: np.ndarray, modes) -> np.ndarray:
    """M_t(A): rows indexed by the modes in t (C-order), columns by the rest."""
    modes = list(modes)
    rest = [m for m in range(A.ndim) if m not in modes]
    P = np.transpose(A, modes + rest)
    rows = int(np.prod([A.shape[m] for m in modes]))
    return P.reshape(rows, -1)


def unmatricize(M: np.ndarray, modes, shape) -> np.ndarray:
    modes = list(modes)
    rest = [m for m in range(len(shape)) if m not in modes]
    perm = modes + rest
    P = M.reshape([shape[m] for m in perm])
    return np.transpose(P, np.argsort(perm))


def singular_values(A: np.ndarray, modes) -> np.ndarray:
    return np.linalg.svd(matricize(A, modes), compute_uv=False)


def leading_vectors(A: np.ndarray, modes, r: int) -> np.ndarray:
    U, _, _ = np.linalg.svd(matricize(A, modes), full_matrices=False)
    return U[:, :r]


def hsvd_full(A: np.ndarray, tree: Tree, ranks: Dict[int, int]) -> HT:
    """Hierarchical SVD of a full tensor (Section 3.3, steps 1-3 for a
    tensor that is not yet in HT format)."""
    Ut = {t: leading_vectors(A, tree.modes(t), ranks[t]) for t in range(1, tree.n_nodes)}
    U = [None] * tree.d
    B = {}
    for t in range(tree.n_nodes):
        if tree.is_leaf(t):
            U[tree.mode(t)] = Ut[t]
            continue
        s1, s2 = tree.sons[t]
        n1 = int(np.prod([A.shape[m] for m in tree.modes(s1)]))
        n2 = int(np.prod([A.shape[m] for m in tree.modes(s2)]))
        if t == 0:
            MD = A.reshape(n1, n2)
            # (B_D)_{j,l} = < M_D(A), (U_t1)_j (x) (U_t2)_l >
            B[0] = np.einsum("ab,aj,bl->jl", MD, Ut[s1], Ut[s2])
        else:
            Ur = Ut[t].reshape(n1, n2, -1)
            # (B_t)_{i,j,l} = < (U_t)_i, (U_s1)_j (x) (U_s2)_l >
            B[t] = np.einsum("abi,aj,bl->ijl", Ur, Ut[s1], Ut[s2])
    return HT(tree, U, B, 0)


def project_root_first(A: np.ndarray, tree: Tree, ranks: Dict[int, int]) -> np.ndarray:
    """prod_{depth p} P_t ... prod_{depth 1} P_t A with P_t the projector on
    the r_t leading left singular vectors of M_t(A) of the ORIGINAL A."""
    P = {t: leading_vectors(A, tree.modes(t), ranks[t]) for t in range(1, tree.n_nodes)}
    X = A.copy()
    for depth in range(1, max(tree.depth) + 1):
        for t in range(1, tree.n_nodes):
            if tree.depth[t] != depth:
                continue
            m = tree.modes(t)
            M = matricize(X, m)
            M = P[t] @ (P[t].T @ M)
            X = unmatricize(M, m, A.shape)
    return X


def best_error_lower_bound(A: np.ndarray, tree: Tree, ranks: Dict[int, int]) -> float:
    """max_t tau_t with tau_t^2 = sum_{i > r_t} sigma_{t,i}^2: every tensor
    of ranks (r_t) is at least this far from A."""
    best = 0.0
    for t in range(1, tree.n_nodes):
        s = singular_values(A, tree.modes(t))
        best = max(best, float(np.sqrt(np.sum(s[ranks[t]:] ** 2))))
    return best
