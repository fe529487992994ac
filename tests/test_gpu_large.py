"""The large single workload at full size: d=128, n=1e5, k=64 per summand
(float32 leaf frames of 1e5 x 128 for the sum, 6.5 GB), transfer tensors with
singular values 10^(-i/16), the sum truncated to rank 64; then ht_entries on
1e6 random multi-indices of the result (Section 3.1, eq. (transfermult)).

Parity: both GPU paths against the oracle's truncation of the same sum
(relative difference norm, Section 3.3), and the GPU entries of the GPU
result against the oracle's level-wise entry recursion of that same tensor
on the first 1e4 indices.  The throughput of ht_entries is printed.
"""
import gc
import sys
import time

import numpy as np
import pytest

import htsynth as S
from oracle import ht_oracle as O

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-6
ENTRY_TOL = 1e-12


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


def test_d128_n1e5_k64_full_size(H):
    import torch
    d, r = 128, 64
    say("case d128_n1e5_k64: generating inputs")
    a, c = S.workload_pair("d128_n1e5_k64")
    say("  oracle truncation to rank 64 (float64)")
    t0 = time.perf_counter()
    X = O.add(O.from_input(a), O.from_input(c))
    T, info = O.truncate(X, mode="fixed", ranks=[r] * (2 * d - 1))
    del X, info
    gc.collect()
    say(f"  oracle took {time.perf_counter() - t0:.1f} s")
    devs = [H.DeviceHT.from_input(a), H.DeviceHT.from_input(c)]
    del a, c
    gc.collect()
    G64 = None
    for prec in (0, 1):
        say(f"  GPU truncation prec={prec}")
        tr = H.Truncator(devs, [1.0, 1.0], mode=H.HT_RANK_FIXED, ranks=[r] * (2 * d - 1), precision=prec,
                         out_frame_dtype=torch.float64, out_transfer_dtype=torch.float64)
        res = tr()
        torch.cuda.synchronize()
        assert res.ranks[1:] == [r] * (2 * d - 2)
        G = to_oracle(res.out)
        err = O.rel_diff(G, T)
        say(f"  prec={prec}: rel err vs oracle {err:.3e}, flags {res.flags}")
        assert err <= (FP64_TOL if prec == 0 else MIXED_TOL)
        if prec == 0:
            G64, out64 = G, res.out
        del tr, res
        gc.collect()
        torch.cuda.empty_cache()
    del T, devs
    gc.collect()

    # entries of the float64 result at 1e6 indices, checked on the first 1e4
    m, m_chk = 1_000_000, 10_000
    idx = S.entry_indices(m, d, 100000, seed=5005)
    idx_dev = torch.from_numpy(idx).cuda()
    H.ht_entries(out64, idx_dev[:1000])                     # plan and first-use costs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got = H.ht_entries(out64, idx_dev)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    say(f"  ht_entries: {m} indices in {dt * 1e3:.1f} ms, {m / dt:.3e} entries/s (rank 64, d=128)")
    got = got.cpu().numpy()
    assert np.all(np.isfinite(got))
    ref = O.entries(G64, idx[:m_chk])
    rel = np.linalg.norm(got[:m_chk] - ref) / np.linalg.norm(ref)
    say(f"  entries vs oracle: relative 2-norm error {rel:.3e} over the first {m_chk} indices")
    assert rel <= ENTRY_TOL
    np.testing.assert_allclose(got[:m_chk], ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
