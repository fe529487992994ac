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


# ------------------------------------------------------------------ config 1 (d=4, n=16, k=4)
@pytest.mark.parametrize("prec", [0, 1])
def test_config1_fixed(H, prec):
    say(f"case config1 fixed prec={prec}")
    a, c = S.config_pair(1)
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
