"""ht_truncate_noalloc, the truncation entry point that allocates nothing,
against ht_truncate on the same inputs, both called through the C ABI.

Two calls in a row share the library's static scratch; the second has a
smaller input, so it runs on what the first left behind.  Each result is
checked against ht_truncate's (the same kernels: they may differ only in the
order of atomic additions) and against the oracle (Section 3.3), and an input
whose workspace exceeds the static array is refused with HT_EWORKSPACE.
"""
import ctypes
import sys

import numpy as np
import pytest

from oracle import ht_oracle as O

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10       # against the oracle, as every float64 parity case
SAME_KERNELS_TOL = 1e-12


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


def rand_ht(rng, d, n, k):
    tr = O.Tree(d)
    U = [rng.standard_normal((n, k)) for _ in range(d)]
    B = {}
    for t in range(tr.n_nodes):
        if not tr.is_leaf(t):
            B[t] = rng.standard_normal((k, k) if t == 0 else (k, k, k))
    return O.HT(tr, U, B, 0)


def run(H, Xs, ranks, noalloc):
    import torch
    devs = [H.DeviceHT.from_arrays(X.d, X.U, [X.B.get(t) for t in range(X.tree.n_nodes)], 0) for X in Xs]
    tr = H.Truncator(devs, [1.0, 1.0], mode=H.HT_RANK_FIXED, ranks=ranks, precision=H.HT_PREC_FP64,
                     out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64, want_sigma=True,
                     noalloc=noalloc)
    res = tr()
    torch.cuda.synchronize()
    U, B, s = res.out.to_host()
    return O.HT(O.Tree(Xs[0].d), U, B, s), res


def test_noalloc_two_calls_then_smaller(H):
    rng = np.random.default_rng(20240611)
    # (d, n, k per summand, target rank): about 10 MiB of workspace, then 0.1 MiB
    for d, n, k, r in [(8, 500, 16, 16), (4, 16, 4, 3)]:
        say(f"case noalloc d={d} n={n} k={k}+{k} -> {r}")
        A, C = rand_ht(rng, d, n, k), rand_ht(rng, d, n, k)
        ranks = [r] * (2 * d - 1)
        ref, _ = O.truncate(O.add(A, C), mode="fixed", ranks=ranks)
        G0, res0 = run(H, [A, C], ranks, noalloc=False)
        G1, res1 = run(H, [A, C], ranks, noalloc=True)
        e_same = O.rel_diff(G1, G0)
        e_or = O.rel_diff(G1, ref)
        say(f"  noalloc vs ht_truncate {e_same:.3e}, vs oracle {e_or:.3e}, flags {res1.flags}")
        assert e_same <= SAME_KERNELS_TOL
        assert e_or <= FP64_TOL
        assert O.rel_diff(G0, ref) <= FP64_TOL
        assert res1.ranks == res0.ranks
        assert res1.flags == res0.flags
        np.testing.assert_allclose(res1.sigma_dev.cpu().numpy(), res0.sigma_dev.cpu().numpy(), rtol=0,
                                   atol=1e-13)


def test_noalloc_refuses_oversized_input(H):
    """A truncation whose workspace exceeds the static array returns
    HT_EWORKSPACE before anything is enqueued (host-only descriptors)."""
    L = H.lib()
    ctx = H.ht_create_context()
    d, n, k = 16, 1000, 32                     # about 165 MiB of workspace
    nn = 2 * d - 1
    nar = (ctypes.c_int64 * d)(*([n] * d))
    rk = (ctypes.c_int32 * nn)(*([k] * nn))
    rk[0] = 1
    desc = H.HtDesc(d, ctypes.cast(nar, ctypes.POINTER(ctypes.c_int64)),
                    ctypes.cast(rk, ctypes.POINTER(ctypes.c_int32)), H.HT_F64, H.HT_F64, None, None, None, 0)
    X = (H.HtDesc * 2)(desc, desc)
    rr = (ctypes.c_int32 * nn)(*([k] * nn))
    opts = H.HtTruncOpts(H.HT_RANK_FIXED, ctypes.cast(rr, ctypes.POINTER(ctypes.c_int32)), 0.0, 1, 0,
                         H.HT_PREC_FP64)
    need = ctypes.c_size_t(0)
    assert L.ht_truncate_workspace(None, X, 2, ctypes.byref(opts), ctypes.byref(need)) == 0
    assert need.value > H.NOALLOC_SCRATCH_BYTES
    st = L.ht_truncate_noalloc(ctx.h, X, None, 2, ctypes.byref(opts), None, None, None, None, None, None)
    assert st == 3, st                         # HT_EWORKSPACE
    assert b"static scratch" in L.ht_last_error()
