"""Pins of the oracle's operator application and truncated solvers
(oracle/operators.py) to facts outside the code under test: the full
matrix-vector product, Kronecker products written out with numpy.kron, mode
products, and the exact solution of a small SPD system by
numpy.linalg.solve."""
import numpy as np
import pytest

from oracle import ht_oracle as O
from oracle import operators as OP


def rand_ht(rng, d, n, ranks, rows=None):
    tr = O.Tree(d)
    U, B = [None] * d, {}
    for t in range(tr.n_nodes):
        if tr.is_leaf(t):
            mu = tr.mode(t)
            U[mu] = rng.standard_normal(((rows or n)[mu], ranks[t]))
        else:
            s1, s2 = tr.sons[t]
            B[t] = rng.standard_normal((ranks[s1], ranks[s2]) if t == 0 else (ranks[t], ranks[s1], ranks[s2]))
    return O.HT(tr, U, B, 0)


def test_apply_equals_matrix_vector_product():
    """Lemma (operator) against (L as a matrix) x vec(A) on a random
    H-operator with uneven ranks and mode sizes."""
    rng = np.random.default_rng(1)
    d, n = 3, [3, 2, 4]
    L = rand_ht(rng, d, n, [1, 2, 3, 2, 3, 2], rows=[m * m for m in n])
    A = rand_ht(rng, d, n, [1, 2, 2, 3, 2, 2])
    C = OP.apply(L, A)
    Lm = OP.operator_matrix(L, n)
    ref = (Lm @ O.full(A).reshape(-1)).reshape(n)
    np.testing.assert_allclose(O.full(C), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert C.ranks() == [1] + [a * b for a, b in zip(L.ranks()[1:], A.ranks()[1:])]


def test_kron_sum_operator_is_the_kronecker_sum():
    rng = np.random.default_rng(2)
    n = [3, 2, 4, 2]
    mats = [rng.standard_normal((m, m)) for m in n]
    L = OP.kron_sum_operator(mats)
    ref = np.zeros((int(np.prod(n)),) * 2)
    for mu in range(len(n)):
        term = np.ones((1, 1))
        for nu in range(len(n)):
            term = np.kron(term, mats[mu] if nu == mu else np.eye(n[nu]))
        ref += term
    np.testing.assert_allclose(OP.operator_matrix(L, n), ref, atol=1e-14)


def test_apply_kron_sum_is_a_sum_of_mode_products():
    """A non-symmetric Kronecker sum fixes the orientation: (L A)[.., j, ..]
    = sum_mu sum_i M_mu[j, i] A[.., i, ..]."""
    rng = np.random.default_rng(3)
    d, n = 4, [3, 4, 2, 3]
    mats = [rng.standard_normal((m, m)) for m in n]
    A = rand_ht(rng, d, n, [1] + [2] * (2 * d - 2))
    Af = O.full(A)
    ref = np.zeros_like(Af)
    for mu in range(d):
        ref += np.moveaxis(np.tensordot(mats[mu], Af, axes=([1], [mu])), 0, mu)
    C = OP.apply(OP.kron_sum_operator(mats), A)
    np.testing.assert_allclose(O.full(C), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def spd_system(rng, d, n, lo=1.0, hi=3.0):
    mats = []
    for m in n:
        q, _ = np.linalg.qr(rng.standard_normal((m, m)))
        mats.append((q * rng.uniform(lo, hi, size=m)[None, :]) @ q.T / d)
    return mats


def test_cg_reaches_the_exact_solution():
    """Algorithm (CG) with a truncation that keeps every direction above
    1e-14 solves a small SPD Kronecker-sum system to the accuracy of
    numpy.linalg.solve on its full matrix."""
    rng = np.random.default_rng(4)
    d, n = 3, [4, 3, 4]
    mats = spd_system(rng, d, n)
    Aop = OP.kron_sum_operator(mats)
    B = rand_ht(rng, d, n, [1] + [2] * (2 * d - 2))
    x = np.linalg.solve(OP.operator_matrix(Aop, n), O.full(B).reshape(-1))
    X, steps = OP.cg(Aop, B, OP.truncation("tol", eps=1e-14), eps=1e-13 * np.sqrt(O.inner(B, B)),
                     max_steps=200)
    err = np.linalg.norm(O.full(X).reshape(-1) - x) / np.linalg.norm(x)
    assert err <= 1e-10, (err, steps)


def test_richardson_reaches_the_exact_solution():
    """Algorithm (richardson) with omega = 2 / (lambda_min + lambda_max)
    contracts by (kappa - 1) / (kappa + 1) per step."""
    rng = np.random.default_rng(5)
    d, n = 3, [3, 4, 3]
    mats = spd_system(rng, d, n, 1.0, 2.0)
    Aop = OP.kron_sum_operator(mats)
    Lm = OP.operator_matrix(Aop, n)
    ev = np.linalg.eigvalsh(Lm)
    omega = 2.0 / (ev[0] + ev[-1])
    B = rand_ht(rng, d, n, [1] + [2] * (2 * d - 2))
    x = np.linalg.solve(Lm, O.full(B).reshape(-1))
    X = OP.richardson(Aop, B, B, omega, OP.truncation("tol", eps=1e-14), steps=80)
    err = np.linalg.norm(O.full(X).reshape(-1) - x) / np.linalg.norm(x)
    rate = (ev[-1] - ev[0]) / (ev[-1] + ev[0])
    assert err <= max(1e-10, 10 * rate ** 80), err


def test_planted_operator_orientation_mistake_is_caught():
    """A copy of apply that contracts the operator's row index instead of its
    column index (L^T A) must fail the mode-product pin."""
    rng = np.random.default_rng(6)
    d, n = 3, [3, 3, 3]
    mats = [rng.standard_normal((m, m)) for m in n]
    A = rand_ht(rng, d, n, [1] + [2] * (2 * d - 2))
    L = OP.kron_sum_operator(mats)
    bad = O.HT(L.tree, [u.reshape(m, m, -1).transpose(1, 0, 2).reshape(m * m, -1) for u, m in zip(L.U, n)],
               L.B, 0)
    Af = O.full(A)
    ref = sum(np.moveaxis(np.tensordot(mats[mu], Af, axes=([1], [mu])), 0, mu) for mu in range(d))
    assert not np.allclose(O.full(OP.apply(bad, A)), ref, atol=1e-8)
