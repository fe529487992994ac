"""Parity of the batched truncation (ht_truncate_batched, through the C ABI)
with the FP64 oracle, problem by problem.

The batched workload: 256 independent sums A_b + C_b, d ~ U{4..32},
n ~ U[100, 4096], k ~ U{8..48}, N(0,1) float32 frames and transfer tensors,
each truncated back to its own k in the mixed path.  The whole batch runs in
one call; a sample of its problems (the oracle takes about a second each) is
compared with the oracle's truncation of the same sums, and every problem is
checked for its ranks and flags.  A second batch mixes rank modes, precisions,
dtypes and summand counts at small sizes, all of it checked.
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


def dev_of(H, X, fdt):
    Bl = [X.B.get(t) for t in range(X.tree.n_nodes)]
    return H.DeviceHT.from_arrays(X.d, X.U, Bl, X.log2_scale, frame_dtype=fdt, transfer_dtype=fdt)


def test_batched_workload_256(H):
    import torch
    meta = S.batched_meta()
    say(f"case batched workload: {len(meta)} problems, mixed precision, fixed ranks k")
    problems, host = [], []
    for m in meta:
        a = S.make_tensor(2 * m["seed_base"], m["d"], m["n"], m["k"], dtype=np.float32)
        c = S.make_tensor(2 * m["seed_base"] + 1, m["d"], m["n"], m["k"], dtype=np.float32)
        da = H.DeviceHT.from_input(a, frame_dtype=torch.float32, transfer_dtype=torch.float32)
        dc = H.DeviceHT.from_input(c, frame_dtype=torch.float32, transfer_dtype=torch.float32)
        nn = 2 * m["d"] - 1
        problems.append(dict(Xs=[da, dc], mode=H.HT_RANK_FIXED, ranks=[m["k"]] * nn, precision=H.HT_PREC_MIXED,
                             out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64))
        host.append((a, c))
    say("  inputs on the device")
    bt = H.BatchTruncator(problems, want_sigma=True)
    res = bt()
    torch.cuda.synchronize()
    say("  batch done")
    for b, (m, r) in enumerate(zip(meta, res)):
        assert r.ranks[1:] == [m["k"]] * (2 * m["d"] - 2), b
        assert not (r.flags & H.HT_FLAG_NONFINITE), b
    # the oracle on every 8th problem (32 of 256, all d, n, k ranges) and the last one
    sample = list(range(0, 256, 8)) + [255]
    worst = 0.0
    for b in sample:
        m = meta[b]
        A, C = O.from_input(host[b][0]), O.from_input(host[b][1])
        T, info = O.truncate(O.add(A, C), mode="fixed", ranks=[m["k"]] * (2 * m["d"] - 1))
        err = O.rel_diff(to_oracle(res[b].out), T)
        worst = max(worst, err)
        say(f"  problem {b} d={m['d']} n={m['n']} k={m['k']}: rel err {err:.3e}")
        assert err <= MIXED_TOL, b
        sig = res[b].sigma_dev.cpu().numpy()
        for t in (1, 2, 2 * m["d"] - 2):
            ref = info["sigma"][t] / info["norm_units"]
            np.testing.assert_allclose(sig[t][:m["k"]], ref[:m["k"]], atol=1e-6)
    say(f"  worst sampled rel err {worst:.3e}")


def rand_ht(rng, d, n, ranks):
    tr = O.Tree(d)
    U = [None] * d
    B = {}
    for t in range(tr.n_nodes):
        if tr.is_leaf(t):
            U[tr.mode(t)] = rng.standard_normal((n[tr.mode(t)], ranks[t]))
        else:
            s1, s2 = tr.sons[t]
            B[t] = rng.standard_normal((ranks[s1], ranks[s2]) if t == 0 else (ranks[t], ranks[s1], ranks[s2]))
    return O.HT(tr, U, B, 0)


def test_batched_mixed_problems(H):
    """Rank modes, precisions, frame dtypes, 1-3 summands, d = 2 and odd d in one batch."""
    import torch
    say("case batched mixed problems")
    rng = np.random.default_rng(21)
    problems, refs = [], []
    specs = [  # d, n_in, mode, precision, float32 frames
        (2, 2, "fixed", 0, False), (3, 1, "tol", 1, True), (4, 2, "fixed", 1, True), (5, 3, "fixed", 0, False),
        (7, 2, "tol", 0, False), (9, 2, "fixed", 1, False), (6, 1, "fixed", 0, True), (13, 2, "tol", 1, True),
        (4, 2, "tol", 0, False), (8, 3, "fixed", 1, True),
    ]
    for i, (d, n_in, mode, prec, f32) in enumerate(specs):
        tr = O.Tree(d)
        nn = 2 * d - 1
        n = [int(x) for x in rng.integers(5, 300, size=d)]
        k = int(rng.integers(2, 12))
        Xs = []
        for c in range(n_in):
            rk = [1] + [k] * (nn - 1)
            X = rand_ht(rng, d, n, rk)
            if f32:   # the oracle sees the float32 values the device holds
                X.U = [u.astype(np.float32).astype(np.float64) for u in X.U]
                X.B = {t: (b if t == 0 else b.astype(np.float32).astype(np.float64)) for t, b in X.B.items()}
            Xs.append(X)
        coef = [float(x) for x in rng.uniform(-2, 2, size=n_in)]
        Y = Xs[0].copy()
        Y = O.add(Xs[0], Xs[1], coef[0], coef[1]) if n_in >= 2 else O.add(Xs[0], Xs[0], coef[0], 0.0)
        if n_in == 3:
            Y = O.add(Y, Xs[2], 1.0, coef[2])
        fdt = torch.float32 if f32 else torch.float64
        devs = [dev_of(H, X, fdt) for X in Xs]
        r = int(max(1, k + int(rng.integers(-3, 3)))) if mode == "fixed" else 0
        if mode == "fixed":
            T, _ = O.truncate(Y, mode="fixed", ranks=[1] + [r] * (nn - 1))
            problems.append(dict(Xs=devs, coef=coef, mode=H.HT_RANK_FIXED, ranks=[1] + [r] * (nn - 1),
                                 precision=prec, out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64))
        else:
            T, _ = O.truncate(Y, mode="tol", eps=0.3, relative=True)
            problems.append(dict(Xs=devs, coef=coef, mode=H.HT_RANK_TOL, eps=0.3, relative=True, precision=prec,
                                 out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64))
        refs.append((T, prec, d, n_in, mode))
    res = H.BatchTruncator(problems)()
    torch.cuda.synchronize()
    for i, (r, (T, prec, d, n_in, mode)) in enumerate(zip(res, refs)):
        err = O.rel_diff(to_oracle(r.out), T)
        say(f"  problem {i} d={d} summands={n_in} {mode} prec={prec}: rel err {err:.3e}")
        assert err <= (FP64_TOL if prec == 0 else MIXED_TOL), i


def test_batched_single_matches_truncate(H):
    """A batch of one gives the result of ht_truncate on the same sum."""
    import torch
    say("case batch of one vs ht_truncate")
    a, c = S.workload_pair("d16_n1000_k32", d=8, n=500)
    da = H.DeviceHT.from_input(a)
    dc = H.DeviceHT.from_input(c)
    nn = 2 * 8 - 1
    kw = dict(mode=H.HT_RANK_FIXED, ranks=[20] * nn, precision=H.HT_PREC_FP64, out_frame_dtype=torch.float64,
              out_transfer_dtype=torch.float64)
    one = H.Truncator([da, dc], [1.0, -0.5], **kw)()
    bat = H.BatchTruncator([dict(Xs=[da, dc], coef=[1.0, -0.5], **kw)])()[0]
    torch.cuda.synchronize()
    assert O.rel_diff(to_oracle(bat.out), to_oracle(one.out)) <= FP64_TOL
    assert bat.ranks == one.ranks and bat.scale_dev.item() == one.scale_dev.item()
