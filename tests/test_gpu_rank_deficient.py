"""Truncation of tensors whose frames are rank-deficient and ill-conditioned
(Section 3.4 orthogonalises every frame; here n_mu < k_mu, so each leaf
frame has a null space, and its nonzero singular values span up to ten
decades).  Such frames arise in every operator application with n_mu small
(Lemma (operator) multiplies the ranks), and an unshifted first Cholesky
sweep can return an unbounded inverse factor on them.

Each case is checked against the full tensor written out (a property of
the result, not of any one implementation): the truncation to relative
accuracy eps must stay within eps of X, and truncating at full rank must
reproduce X, both up to the resolution of the Gramian method.  A frame
direction with singular value sigma enters the Gramians as sigma^2, so
below about sqrt(K u) sigma_max it cannot be told from the rounding of the
k - n null directions that the library's k-column factor carries (the
oracle's Householder QR has only n columns); cutting the leaf to rank n
can then lose such a direction, an error of at most about sqrt(K u) =
4e-8.  The gates are 1e-7 (float64) and 1e-6 (mixed), far below what an
unbounded factor gives (errors of order 1 and above).
"""
import sys

import numpy as np
import pytest

from oracle import ht_oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1708_03340_amd as H
    H.lib()
    return H


def graded_frame(rng, n, k, r, decades):
    """n x k of rank r with singular values 10^0 .. 10^-decades."""
    U, _ = np.linalg.qr(rng.standard_normal((n, r)))
    V, _ = np.linalg.qr(rng.standard_normal((k, r)))
    return (U * 10.0 ** -np.linspace(0.0, decades, r)) @ V.T


def case(rng, d, n, k):
    tr = O.Tree(d)
    U = [graded_frame(rng, n, k, int(rng.integers(max(1, n - 3), n + 1)), float(rng.uniform(0, 10)))
         for _ in range(d)]
    B = {t: rng.standard_normal((k, k) if t == 0 else (k, k, k)) for t in range(tr.n_nodes) if not tr.is_leaf(t)}
    return O.HT(tr, U, B, 0)


def to_oracle(dev):
    U, B, s = dev.to_host()
    return O.HT(O.Tree(dev.d), U, B, s)


@pytest.mark.parametrize("prec", [0, 1])
def test_rank_deficient_frames(H, prec):
    import torch
    f64 = torch.float64
    d, k, nn = 4, 12, 7
    rng = np.random.default_rng(4242 + prec)
    worst_tol = worst_full = 0.0
    precision = H.HT_PREC_FP64 if prec == 0 else H.HT_PREC_MIXED
    eps = 1e-6 if prec == 0 else 1e-4
    full_gate = 1e-7 if prec == 0 else 1e-6
    for trial in range(24):
        n = int(rng.choice([6, 8, 10]))
        X = case(rng, d, n, k)
        say(f"case rank-deficient frames prec {prec} trial {trial}: d={d} n={n} k={k}")
        Xf = O.full(X)
        nx = np.linalg.norm(Xf)
        dev = H.DeviceHT.from_arrays(d, X.U, [X.B.get(t) for t in range(nn)], 0, frame_dtype=f64,
                                     transfer_dtype=f64)
        tol = H.Truncator([dev], [1.0], mode=H.HT_RANK_TOL, eps=eps, relative=True, precision=precision,
                          out_frame_dtype=f64, out_transfer_dtype=f64)
        res = tol()
        torch.cuda.synchronize()
        e_tol = np.linalg.norm(O.full(to_oracle(res.out)) - Xf) / nx
        full = H.Truncator([dev], [1.0], mode=H.HT_RANK_FIXED, ranks=[k] * nn, precision=precision,
                           out_frame_dtype=f64, out_transfer_dtype=f64)
        res2 = full()
        torch.cuda.synchronize()
        e_full = np.linalg.norm(O.full(to_oracle(res2.out)) - Xf) / nx
        say(f"  tol {eps:g}: error {e_tol:.3e} ranks {res.ranks}; full rank: error {e_full:.3e}")
        worst_tol, worst_full = max(worst_tol, e_tol), max(worst_full, e_full)
        assert e_tol <= 1.01 * eps + full_gate
        assert e_full <= full_gate
    say(f"  worst: tol {worst_tol:.3e}, full {worst_full:.3e}")
