"""Parity of the HIP path (called through the C ABI) with the FP64 oracle.

Gates (derived in the design notes): FP64 path rel. error <= 1e-10, mixed
path <= 1e-6, both measured as ||X_gpu - X_oracle|| / ||X_oracle|| through the
orthogonalised HT difference.  Ranks chosen by the tolerance rule must equal
the oracle's; sigma / ||A|| per node must agree.
"""
import sys

import numpy as np
import pytest

import htsynth as S
from oracle import ht_oracle as O

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-6
# The d=64, n=1e4, k=64 recipe (N(0,1) frames, spectra 0.9^i, tolerance 1e-6) cuts
# where lambda_r / lambda_1 ~ 3e-14 with relative gaps ~2e-15: the FP64
# Gramians cannot resolve the kept subspace there, and the oracle itself moves
# by 1.4e-9 (d=16) / 2.1e-9 (d=64) when its inputs change by 1e-16.  The FP64
# gate for that recipe is five times the oracle's own spread
# (tests/test_oracle_noise.py measures it on the CPU; the same workload at
# fixed rank 64 is held to FP64_TOL).
FP64_TOL_CUT_AT_NOISE = 1e-8


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


def to_oracle(dev):
    U, B, s = dev.to_host()
    return O.HT(O.Tree(dev.d), U, B, s)


def rand_ht(rng, d, n, ranks):
    tr = O.Tree(d)
    ns = [int(n)] * d if np.isscalar(n) else list(n)
    U = [None] * d
    B = {}
    for t in range(tr.n_nodes):
        if tr.is_leaf(t):
            U[tr.mode(t)] = rng.standard_normal((ns[tr.mode(t)], ranks[t]))
        else:
            s1, s2 = tr.sons[t]
            shape = (ranks[s1], ranks[s2]) if t == 0 else (ranks[t], ranks[s1], ranks[s2])
            B[t] = rng.standard_normal(shape)
    return O.HT(tr, U, B, 0)


def dev_of(H, X, fdt=None, tdt=None):
    import torch
    fdt = fdt or torch.float64
    tdt = tdt or torch.float64
    Bl = [X.B.get(t) for t in range(X.tree.n_nodes)]
    return H.DeviceHT.from_arrays(X.d, X.U, Bl, X.log2_scale, frame_dtype=fdt, transfer_dtype=tdt)


def run_trunc(H, Xs_or, coef, prec, mode, ranks=None, eps=0.0, max_rank=0, fdt=None, want_sigma=True):
    import torch
    devs = [dev_of(H, X, fdt, fdt) for X in Xs_or]
    tr = H.Truncator(devs, coef, mode=mode, ranks=ranks, eps=eps, max_rank=max_rank, precision=prec,
                     out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64, want_sigma=want_sigma)
    res = tr()
    torch.cuda.synchronize()
    return res


def oracle_sum(Xs, coef):
    Y = Xs[0].copy()
    Y = O.add(Xs[0], Xs[1], coef[0], coef[1]) if len(Xs) == 2 else Xs[0]
    return Y


# ------------------------------------------------------------------ workload d=4, n=16, k=4
@pytest.mark.parametrize("prec", [0, 1])
def test_d4_n16_k4_fixed(H, prec):
    say(f"case d4_n16_k4 fixed prec={prec}")
    a, c = S.workload_pair("d4_n16_k4")
    A, C = O.from_input(a), O.from_input(c)
    X = O.add(A, C)
    T, info = O.truncate(X, mode="fixed", ranks=[4] * 7)
    res = run_trunc(H, [A, C], [1.0, 1.0], prec, H.HT_RANK_FIXED, ranks=[4] * 7)
    G = to_oracle(res.out)
    err = O.rel_diff(G, T)
    say(f"  rel err {err:.3e} flags {res.flags}")
    assert err <= (FP64_TOL if prec == 0 else MIXED_TOL)
    assert res.ranks[1:] == [4] * 6
    sig = res.sigma_dev.cpu().numpy()
    for t in range(1, 7):
        ref = info["sigma"][t] / info["norm_units"]
        np.testing.assert_allclose(sig[t][:8], ref[:8], atol=1e-12 if prec == 0 else 1e-6)


@pytest.mark.parametrize("prec", [0, 1])
def test_orthogonalize(H, prec):
    say(f"case orthogonalize d=5 prec={prec}")
    import torch
    rng = np.random.default_rng(7)
    X = rand_ht(rng, 5, [37, 70, 65, 129, 40], [1, 5, 6, 4, 3, 9, 7, 5, 8])
    dev = dev_of(H, X)
    H.ht_orthogonalize(dev, precision=prec)
    torch.cuda.synchronize()
    G = to_oracle(dev)
    err = O.rel_diff(G, X)
    say(f"  rel err {err:.3e}")
    assert err <= (1e-12 if prec == 0 else 1e-6)
    tr = G.tree
    for t in range(1, tr.n_nodes):
        if tr.is_leaf(t):
            U = G.U[tr.mode(t)]
            np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
        else:
            M = G.B[t].reshape(G.B[t].shape[0], -1)
            np.testing.assert_allclose(M @ M.T, np.eye(M.shape[0]), atol=1e-12 if prec == 0 else 1e-6)


def test_gramians(H):
    say("case gramians d=6")
    rng = np.random.default_rng(8)
    X = rand_ht(rng, 6, 50, [1] + [6] * 10)
    Xo = O.orthogonalize(X)
    Gr, g = O.gramians(Xo)
    dev = dev_of(H, Xo)
    bh, sg, units = H.ht_gramians(dev)
    import torch
    torch.cuda.synchronize()
    assert int(units.item()) == g
    for t in range(1, X.tree.n_nodes):
        np.testing.assert_allclose(bh[t].cpu().numpy(), Gr[t], atol=1e-12 * np.abs(Gr[t]).max())
        lam, _ = O.eig_desc(Gr[t])
        np.testing.assert_allclose(sg[t].cpu().numpy() ** 2, lam, atol=1e-12 * lam.max())


def test_entries(H):
    say("case entries d=7")
    import torch
    rng = np.random.default_rng(9)
    X = rand_ht(rng, 7, 33, [1] + [5] * 12)
    X.log2_scale = 3
    idx = S.entry_indices(3000, 7, 33, seed=1)
    ref = O.entries(X, idx)
    out = H.ht_entries(dev_of(H, X), torch.from_numpy(idx))
    got = out.cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_add(H):
    say("case add d=4")
    import torch
    rng = np.random.default_rng(10)
    A = rand_ht(rng, 4, 9, [1, 3, 2, 4, 2, 3, 2])
    C = rand_ht(rng, 4, 9, [1, 2, 3, 1, 5, 2, 2])
    C.log2_scale = -2
    Sg = H.ht_add(dev_of(H, A), dev_of(H, C), 0.5, 3.0)
    torch.cuda.synchronize()
    G = to_oracle(Sg)
    R = O.add(A, C, 0.5, 3.0)
    np.testing.assert_allclose(O.full(G), O.full(R), rtol=1e-14, atol=1e-14 * np.abs(O.full(R)).max())


# ------------------------------------------------------------------ workload d=16, n=1000, k=32, spectrum 10^(-i/8)
@pytest.mark.parametrize("prec", [0, 1])
def test_d16_n1000_k32(H, prec):
    say(f"case d16_n1000_k32 prec={prec}")
    a, c = S.workload_pair("d16_n1000_k32")
    A, C = O.from_input(a), O.from_input(c)
    X = O.add(A, C)
    nn = 2 * 16 - 1
    T, info = O.truncate(X, mode="fixed", ranks=[32] * nn)
    res = run_trunc(H, [A, C], [1.0, 1.0], prec, H.HT_RANK_FIXED, ranks=[32] * nn)
    err = O.rel_diff(to_oracle(res.out), T)
    say(f"  rel err {err:.3e} flags {res.flags}")
    assert err <= (FP64_TOL if prec == 0 else MIXED_TOL)
    # Gramian eigenvalues carry an absolute error of order u ||A||^2, so the
    # squares are compared (sigma near 1e-4 ||A|| is only good to ~1e-8)
    sig = res.sigma_dev.cpu().numpy()
    worst = max(np.max(np.abs(sig[t][:64] ** 2 - (info["sigma"][t] / info["norm_units"]) ** 2))
                for t in range(1, nn))
    say(f"  max |(sigma/||A||)^2 - oracle| {worst:.3e}")
    assert worst <= (1e-13 if prec == 0 else 1e-6)


# ------------------------------------------------------------------ the d=64, n=1e4, k=64 recipe at reduced d and n
def test_d64_recipe_reduced_tolerance(H):
    say("case d64_n1e4_k64 recipe at d=8 n=2000 k=64 tol 1e-6 mixed")
    import torch
    a, c = S.workload_pair("d64_n1e4_k64", d=8, n=2000)
    A, C = O.from_input(a), O.from_input(c)
    X = O.add(A, C)
    T, info = O.truncate(X, mode="tol", eps=1e-6, relative=True)
    devs = [H.DeviceHT.from_input(a), H.DeviceHT.from_input(c)]
    tr = H.Truncator(devs, [1.0, 1.0], mode=H.HT_RANK_TOL, eps=1e-6, relative=True, precision=H.HT_PREC_MIXED,
                     out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64)
    res = tr()
    torch.cuda.synchronize()
    gr = res.ranks
    orr = [1] + [info["ranks"][t] for t in range(1, 15)]
    say(f"  gpu ranks {gr[1:]}\n  oracle ranks {orr[1:]}")
    assert gr[1:] == orr[1:]
    G = to_oracle(res.out)
    err = O.rel_diff(G, T)
    say(f"  rel err vs oracle {err:.3e}; achieved truncation error {O.rel_diff(G, X):.3e}")
    assert err <= MIXED_TOL
    assert O.rel_diff(G, X) <= 1e-6 * (1 + 1e-6) + 2e-7


@pytest.fixture(scope="module")
def d64():
    """The d=64, n=1e4, k=64 workload, its oracle sum and the oracle's
    tolerance-mode truncation (computed once for the full-size cases)."""
    a, c = S.workload_pair("d64_n1e4_k64")
    A, C = O.from_input(a), O.from_input(c)
    X = O.add(A, C)
    T, info = O.truncate(X, mode="tol", eps=1e-6, relative=True)
    return dict(a=a, c=c, A=A, C=C, X=X, T=T, info=info)


@pytest.mark.parametrize("prec", [0, 1])
def test_d64_n1e4_k64_full_size(H, prec, d64):
    """The benchmark's workload at full size: GPU vs oracle on the whole
    truncated tensor (tolerance mode; parity at the oracle's ranks)."""
    say(f"case d64_n1e4_k64 full size prec={prec}")
    import torch
    a, c, T, info = d64["a"], d64["c"], d64["T"], d64["info"]
    devs = [H.DeviceHT.from_input(a), H.DeviceHT.from_input(c)]
    tr = H.Truncator(devs, [1.0, 1.0], mode=H.HT_RANK_TOL, eps=1e-6, relative=True, precision=prec,
                     out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64)
    res = tr()
    torch.cuda.synchronize()
    orr = [info["ranks"][t] for t in range(1, 127)]
    same = sum(int(g == o) for g, o in zip(res.ranks[1:], orr))
    say(f"  ranks equal at {same}/126 nodes; gpu range {min(res.ranks[1:])}..{max(res.ranks[1:])}")
    G = to_oracle(res.out)
    err = O.rel_diff(G, T)
    say(f"  rel err vs oracle {err:.3e}")
    assert same == 126
    assert err <= (FP64_TOL_CUT_AT_NOISE if prec == 0 else MIXED_TOL)


@pytest.mark.parametrize("prec", [0, 1])
def test_d64_n1e4_k64_fixed_r64(H, prec, d64):
    """The same workload truncated to fixed rank 64: no rank decision sits at
    the rounding level, so the float64 path is held to the 1e-10 gate."""
    say(f"case d64_n1e4_k64 full size fixed r=64 prec={prec}")
    import torch
    T, _ = O.truncate(d64["X"], mode="fixed", ranks=[64] * 127)
    devs = [H.DeviceHT.from_input(d64["a"]), H.DeviceHT.from_input(d64["c"])]
    tr = H.Truncator(devs, [1.0, 1.0], mode=H.HT_RANK_FIXED, ranks=[64] * 127, precision=prec,
                     out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64)
    res = tr()
    torch.cuda.synchronize()
    err = O.rel_diff(to_oracle(res.out), T)
    say(f"  rel err vs oracle {err:.3e} flags {res.flags}")
    assert res.ranks[1:] == [64] * 126
    assert err <= (FP64_TOL if prec == 0 else MIXED_TOL)


def test_entries_full_size_rank128(H, d64):
    """ht_entries on the materialised d=64, n=1e4 sum (rank 128 at every
    node): 2e5 indices span 13 chunks of the level-wise evaluation (the last
    one ragged) with Khatri-Rao reductions of 128 x 128 = 16384; every 97th
    index is checked against the oracle's eq. (transfermult) recursion."""
    say("case entries d=64 n=1e4 rank 128, m=2e5")
    import torch
    da, dc = H.DeviceHT.from_input(d64["a"]), H.DeviceHT.from_input(d64["c"])
    Sd = H.ht_add(da, dc, 1.0, 1.0)
    idx = S.entry_indices(200000, 64, 10000, seed=606)
    got = H.ht_entries(Sd, torch.from_numpy(idx)).cpu().numpy()
    sub = np.arange(0, idx.shape[0], 97)
    ref = O.entries(d64["X"], idx[sub])
    rel = np.linalg.norm(got[sub] - ref) / np.linalg.norm(ref)
    say(f"  sampled relative 2-norm error {rel:.3e} over {sub.size} indices")
    assert rel <= 1e-12
    np.testing.assert_allclose(got[sub], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    assert np.all(np.isfinite(got))


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_input_flagged(H, bad):
    """A NaN or Inf in a leaf frame is reported in the flags word
    (HT_FLAG_NONFINITE); the call still completes."""
    say(f"case non-finite input {bad}")
    a, c = S.workload_pair("d4_n16_k4")
    A, C = O.from_input(a), O.from_input(c)
    A.U[2] = A.U[2].copy()
    A.U[2][5, 1] = bad
    res = run_trunc(H, [A, C], [1.0, 1.0], 0, H.HT_RANK_FIXED, ranks=[4] * 7)
    say(f"  flags {res.flags:#x}")
    assert res.flags & H.HT_FLAG_NONFINITE


# ------------------------------------------------------------------ edge cases
def test_d2_eckart_young(H):
    say("case d=2")
    rng = np.random.default_rng(11)
    A = rand_ht(rng, 2, [9, 7], [1, 3, 2])
    C = rand_ht(rng, 2, [9, 7], [1, 2, 4])
    X = O.add(A, C)
    T, _ = O.truncate(X, mode="fixed", ranks=[1, 3, 3])
    res = run_trunc(H, [A, C], [1.0, 1.0], 0, H.HT_RANK_FIXED, ranks=[1, 3, 3])
    assert O.rel_diff(to_oracle(res.out), T) <= FP64_TOL


@pytest.mark.parametrize("d", [3, 5, 7, 13])
def test_odd_d_ragged(H, d):
    say(f"case odd d={d} ragged")
    rng = np.random.default_rng(20 + d)
    nn = 2 * d - 1
    ranks_a = [1] + [int(x) for x in rng.integers(3, 40, size=nn - 1)]
    ranks_c = [1] + [int(x) for x in rng.integers(2, 30, size=nn - 1)]
    ns = [int(x) for x in rng.integers(70, 300, size=d)]
    A = rand_ht(rng, d, ns, ranks_a)
    C = rand_ht(rng, d, ns, ranks_c)
    X = O.add(A, C)
    r = [1] + [int(x) for x in rng.integers(2, 20, size=nn - 1)]
    T, info = O.truncate(X, mode="fixed", ranks=r)
    for prec in (0, 1):
        res = run_trunc(H, [A, C], [0.7, -1.3], prec, H.HT_RANK_FIXED, ranks=r)
        T2, _ = O.truncate(O.add(A, C, 0.7, -1.3), mode="fixed", ranks=r)
        err = O.rel_diff(to_oracle(res.out), T2)
        say(f"  prec {prec} rel err {err:.3e}")
        assert err <= (FP64_TOL if prec == 0 else MIXED_TOL)


def test_n_smaller_than_rank(H):
    """n = 3 < K = 8: every leaf frame is rank deficient; the dropped
    directions are flagged and the result still equals the oracle's."""
    say("case n < K")
    rng = np.random.default_rng(12)
    A = rand_ht(rng, 4, 3, [1] + [4] * 6)
    C = rand_ht(rng, 4, 3, [1] + [4] * 6)
    X = O.add(A, C)
    T, _ = O.truncate(X, mode="fixed", ranks=[1] + [2] * 6)
    res = run_trunc(H, [A, C], [1.0, 1.0], 0, H.HT_RANK_FIXED, ranks=[1] + [2] * 6)
    err = O.rel_diff(to_oracle(res.out), T)
    say(f"  rel err {err:.3e} flags {res.flags}")
    assert err <= 1e-9
    assert res.flags & H.HT_FLAG_RANK_DEFICIENT


@pytest.mark.parametrize("prec", [0, 1])
def test_a_plus_a_is_2a(H, prec):
    say(f"case A+A prec={prec}")
    a, _ = S.workload_pair("d16_n1000_k32", d=8)
    A = O.from_input(a)
    res = run_trunc(H, [A, A], [1.0, 1.0], prec, H.HT_RANK_FIXED, ranks=[32] * 15)
    err = O.rel_diff(to_oracle(res.out), O.add(A, A, 2.0, 0.0))
    say(f"  rel err vs 2A {err:.3e} flags {res.flags}")
    # the Gramian next to the root has a kept eigenvalue at 1e-21 of the
    # largest, below the absolute resolution of any float64 eigensolver
    assert err <= (FP64_TOL if prec == 0 else MIXED_TOL)
    assert res.flags & H.HT_FLAG_RANK_DEFICIENT


def test_zero_partner_and_three_summands(H):
    say("case zero partner, three summands")
    a, c = S.workload_pair("d4_n16_k4")
    A, C = O.from_input(a), O.from_input(c)
    res = run_trunc(H, [A, C], [1.0, 0.0], 0, H.HT_RANK_FIXED, ranks=[4] * 7)
    assert O.rel_diff(to_oracle(res.out), A) <= FP64_TOL
    rng = np.random.default_rng(13)
    E = rand_ht(rng, 4, 16, [1] + [3] * 6)
    X3 = O.add(O.add(A, C, 1.0, 2.0), E, 1.0, -0.5)
    T, _ = O.truncate(X3, mode="fixed", ranks=[1] + [6] * 6)
    res = run_trunc(H, [A, C, E], [1.0, 2.0, -0.5], 0, H.HT_RANK_FIXED, ranks=[1] + [6] * 6)
    assert O.rel_diff(to_oracle(res.out), T) <= FP64_TOL


def test_tolerance_extremes(H):
    say("case eps >= 1 and eps = 0")
    a, c = S.workload_pair("d4_n16_k4")
    A, C = O.from_input(a), O.from_input(c)
    res = run_trunc(H, [A, C], [1.0, 1.0], 0, H.HT_RANK_TOL, eps=2.0)
    assert res.ranks[1:] == [1] * 6
    res = run_trunc(H, [A, C], [1.0, 1.0], 0, H.HT_RANK_TOL, eps=0.0)
    assert O.rel_diff(to_oracle(res.out), O.add(A, C)) <= FP64_TOL
    res = run_trunc(H, [A, C], [1.0, 1.0], 0, H.HT_RANK_TOL, eps=0.0, max_rank=3)
    assert max(res.ranks[1:]) <= 3 and res.flags & H.HT_FLAG_CAPPED


def test_huge_scale(H):
    """Scale exponents far outside float64: the result's scale shifts exactly."""
    say("case huge scale")
    a, c = S.workload_pair("d4_n16_k4")
    A, C = O.from_input(a), O.from_input(c)
    A.log2_scale = C.log2_scale = 3000
    res = run_trunc(H, [A, C], [1.0, 1.0], 0, H.HT_RANK_FIXED, ranks=[4] * 7)
    A.log2_scale = C.log2_scale = 0
    T, _ = O.truncate(O.add(A, C), mode="fixed", ranks=[4] * 7)
    G = to_oracle(res.out)
    G.log2_scale -= 3000
    assert O.rel_diff(G, T) <= FP64_TOL


@pytest.mark.parametrize("k0,k1", [(40, 60), (32, 33), (32, 32), (1, 127), (127, 1)])
def test_unequal_summand_ranks(H, k0, k1):
    """Two summands of leaf ranks k0 and k1.  From a sum of 65 up to 128 the
    leaf Gram matrix of the first CholeskyQR2 sweep is one split-K descriptor
    whose rows from k0 on lie in the second frame's buffer (32 + 32 takes the
    blockwise path).  Float32 and float64 frames, both paths."""
    import torch
    say(f"case summand leaf ranks {k0} + {k1}")
    rng = np.random.default_rng(31 + k0)
    d = 6
    nn = 2 * d - 1
    tr = O.Tree(d)
    # inner ranks within what the sons' ranks allow (rank 1 below rank 1)
    ra = [1] + [k0 if tr.is_leaf(t) else min(24, k0) for t in range(1, nn)]
    rc = [1] + [k1 if tr.is_leaf(t) else min(20, k1) for t in range(1, nn)]
    ns = [int(x) for x in rng.integers(300, 700, size=d)]
    A = rand_ht(rng, d, ns, ra)
    C = rand_ht(rng, d, ns, rc)
    r = [1] + [30] * (nn - 1)
    for fdt in (torch.float64, torch.float32):
        if fdt == torch.float32:   # the oracle sees the float32 values the device holds
            for X in (A, C):
                X.U = [u.astype(np.float32).astype(np.float64) for u in X.U]
                X.B = {t: (b if t == 0 else b.astype(np.float32).astype(np.float64)) for t, b in X.B.items()}
        T, _ = O.truncate(O.add(A, C, 1.0, -0.8), mode="fixed", ranks=r)
        for prec in (0, 1):
            res = run_trunc(H, [A, C], [1.0, -0.8], prec, H.HT_RANK_FIXED, ranks=r, fdt=fdt)
            err = O.rel_diff(to_oracle(res.out), T)
            say(f"  frames {fdt} prec {prec} rel err {err:.3e}")
            assert err <= (FP64_TOL if prec == 0 else MIXED_TOL)
